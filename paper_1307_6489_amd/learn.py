"""Learned gamma/hadron + energy estimator: data, training, evaluation.

Pipeline (every per-image step on the GPU kernels of librta):
  1. images      seeded gamma / hadron charge images from the generator
                 (gammas: one narrow ellipse, size = 1000 p.e. x E/TeV with E
                 log-uniform in 0.03..100 TeV; hadrons: 1..4 broad blobs),
  2. features    rta_clean -> rta_hillas -> rta_features on the device,
  3. tables      feature standardisation and box-cut tables (host statistics
                 of the training features),
  4. training    rta_mlp_train_step (BF16 MFMA forward / backward + Adam),
  5. evaluation  rta_classify with and without the network on a held-out
                 seed: hadron acceptance at equal gamma efficiency, energy
                 resolution, and the throughput cost of the network.

Run ``python -m paper_1307_6489_amd.learn --help`` for the full-size job.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

import paper_1307_6489_amd as rta
from paper_1307_6489_amd import boxcut


def init_params(seed):
    """He-normal weights, zero biases, packed as the network expects."""
    rng = np.random.default_rng(seed)
    parts = []
    for n_in, n_out in ((10, 64), (64, 64), (64, 64), (64, 2)):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / n_in), size=(n_in, n_out)).reshape(-1))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts).astype(np.float32)


HADRONS = ("blobs", "single")


def draw_cfg(cam, hadrons="blobs"):
    """Generator settings of the gamma / hadron images.  hadrons="blobs":
    1..4 broad blobs (width 0.06..0.15 m, length 1..2 x width); "single":
    one ellipse whose width (0.03..0.09 m) and length / width (1..2.5)
    overlap the gammas' (0.02..0.06 m, 1.5..4), so that no single cut
    separates the two populations."""
    import dl0sim
    if hadrons not in HADRONS:
        raise ValueError("hadrons must be one of %s" % (HADRONS,))
    cfg = dl0sim.draw_cfg_plain(cam.n_samp)
    if hadrons == "single":
        cfg.had_blobs_max = 1
        cfg.had_width_min, cfg.had_width_max = 0.03, 0.09
        cfg.had_lw_min, cfg.had_lw_max = 1.0, 2.5
    return cfg


def image_features(cam, n, seed, dev, chunk=50_000, first_event=0, log=None, hadrons="blobs"):
    """Generate n charge images and reduce them on the GPU to Hillas records
    and network features.  Returns dict of numpy arrays."""
    import torch
    import dl0sim
    gcam = rta.Camera.from_type(cam)
    cfg = draw_cfg(cam, hadrons)
    feats, recs, labels, energies = [], [], [], []
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        sh = dl0sim.draw_gamma_hadron(cfg, seed, first_event + c0, m)
        ids = np.arange(first_event + c0, first_event + c0 + m, dtype=np.uint64)
        d, t = dl0sim.render_images(cam, sh, seed, event_ids=ids)
        D = torch.from_numpy(d).to(dev)
        T = torch.from_numpy(t).to(dev)
        mask = rta.clean(gcam, D)
        rec = rta.hillas_q8(gcam, D, T, mask)
        x = rta.features(rec)
        feats.append(x.cpu().numpy())
        recs.append(rta.records(rec))
        labels.append((sh["kind"] == 1).astype(np.float32))
        energies.append(np.log10(sh["energy_tev"]).astype(np.float32))
        if log:
            log("images %d / %d (seed %d)" % (c0 + m, n, seed))
    return {"x": np.concatenate(feats), "rec": np.concatenate(recs), "label": np.concatenate(labels),
            "log10e": np.concatenate(energies)}


def usable(x, rec):
    return np.all(np.isfinite(x), 1) & ((rec["flags"] & rta.FLAG_HILLAS_INVALID) == 0)


def train(data, dev, epochs=10, batch=4096, lr=1e-3, seed=3, log=None):
    """Fit standardisation and box cuts, then train the network on the GPU."""
    import torch
    x, rec, lab, e = data["x"], data["rec"], data["label"], data["log10e"]
    ok = usable(x, rec)
    xt, lt, et = x[ok], lab[ok], e[ok]
    mean = xt.mean(0)
    std = xt.std(0) + 1e-6
    g = lt > 0.5
    bc = boxcut.fit(xt[g], xt[~g], et[g])
    net = rta.Mlp(max_batch=batch, lr=lr)
    net.set_params(init_params(seed), mean, std)
    X = torch.from_numpy(np.ascontiguousarray(xt)).to(dev)
    L = torch.from_numpy(np.ascontiguousarray(lt)).to(dev)
    E = torch.from_numpy(np.ascontiguousarray(et)).to(dev)
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, device=dev)
    n = len(xt)
    history = []
    t0 = time.time()
    steps = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(dev)
        for s in range(0, n - batch + 1, batch):
            net.train_step(X, L, E, loss_out=loss, rows=perm[s:s + batch])
            steps += 1
        history.append(float(loss.cpu()[0]))
        if log:
            log("epoch %d: loss %.4f" % (ep, history[-1]))
    torch.cuda.synchronize()
    train_s = time.time() - t0
    # network threshold at the box cuts' target efficiency, on training gammas
    cls = rta.classify(net, bc, torch.from_numpy(rec[ok][g].view(np.float32).reshape(-1, 16).copy()).to(dev))
    boxcut.set_score_cut(bc, cls[:, 0].cpu().numpy())
    return net, bc, {"loss_history": history, "train_seconds": train_s, "steps": steps, "n_train": int(n),
                     "batch": batch, "epochs": epochs}


def binomial_ci(k, n):
    p = k / max(n, 1)
    return p, math.sqrt(max(p * (1 - p), 1.0 / max(n, 1)) / max(n, 1))


def evaluate(net, bc, data, dev, timing_reps=20):
    """Held-out comparison at equal gamma efficiency (the network's threshold
    is moved to the box cuts' held-out gamma efficiency)."""
    import torch
    rec, lab, e = data["rec"], data["label"], data["log10e"]
    R = torch.from_numpy(np.ascontiguousarray(rec).view(np.float32).reshape(-1, 16).copy()).to(dev)
    box = rta.classify(None, bc, R).cpu().numpy()
    net_out = rta.classify(net, bc, R).cpu().numpy()
    valid = (rec["flags"] & rta.FLAG_HILLAS_INVALID) == 0
    g = (lab > 0.5) & valid
    h = (lab < 0.5) & valid
    eff_box = float(np.mean(box[g, 2] > 0.5))
    acc_box = int(np.sum(box[h, 2] > 0.5))
    # equal efficiency: threshold on the network score at the box efficiency
    sg = np.sort(net_out[g, 0])
    thr = sg[int(np.floor((1.0 - eff_box) * len(sg)))]
    eff_net = float(np.mean(net_out[g, 0] >= thr))
    acc_net = int(np.sum(net_out[h, 0] >= thr))
    pb, sb = binomial_ci(acc_box, int(h.sum()))
    pn, sn = binomial_ci(acc_net, int(h.sum()))
    res_box = float(np.std(box[g, 1] - e[g]))
    res_net = float(np.std(net_out[g, 1] - e[g]))
    # throughput cost of the network in the classification kernel
    n = R.shape[0]
    ts = {}
    for name, m in (("box_only", None), ("network", net)):
        rta.classify(m, bc, R)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(timing_reps):
            rta.classify(m, bc, R)
        b.record()
        b.synchronize()
        ts[name] = a.elapsed_time(b) / timing_reps
    return {
        "n_gamma": int(g.sum()), "n_hadron": int(h.sum()),
        "gamma_eff_box": eff_box, "gamma_eff_network": eff_net,
        "hadron_acc_box": pb, "hadron_acc_box_err": sb,
        "hadron_acc_network": pn, "hadron_acc_network_err": sn,
        "log10e_rms_linear_fit": res_box, "log10e_rms_network": res_net,
        "fallback_fraction": float(np.mean(net_out[valid, 3])),
        "classify_ms_box_only": ts["box_only"], "classify_ms_network": ts["network"],
        "records": int(n),
        "classify_records_per_s_network": n / (ts["network"] * 1e-3),
    }


def main():
    import torch
    import dl0sim
    ap = argparse.ArgumentParser(description="train and evaluate the gamma/hadron + energy network")
    ap.add_argument("--train", type=int, default=2_000_000)
    ap.add_argument("--test", type=int, default=200_000)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--out", type=str, default="")
    ap.add_argument("--hadrons", choices=HADRONS, default="blobs",
                    help="hadron images: 1..4 broad blobs, or single ellipses overlapping the gammas in width "
                         "and length")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    cam = dl0sim.camera_c0()
    t0 = time.time()
    say = lambda s: print(s, flush=True)
    tr = image_features(cam, args.train, 3, dev, log=say, hadrons=args.hadrons)
    te = image_features(cam, args.test, 4, dev, log=say, hadrons=args.hadrons)
    print("features in %.1f s" % (time.time() - t0), flush=True)
    net, bc, info = train(tr, dev, epochs=args.epochs, log=say)
    res = evaluate(net, bc, te, dev)
    res.update(info)
    res["hadrons"] = args.hadrons
    print(json.dumps(res), flush=True)
    if args.out:
        np.savez(args.out, params=net.get_params(), mean=tr["x"][usable(tr["x"], tr["rec"])].mean(0))
        with open(args.out + ".json", "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
