/*
 * CPU ORACLE — test infrastructure only.
 *
 * A plain, slow, obviously-correct FP64 / int64 implementation of the
 * low-level reconstruction that the real-time analysis applies to every camera
 * event (calibration of the DL0 data, then the image parameters that feed
 * gamma/hadron separation, energy and direction; Section 4.1 of the paper,
 * with the reduced-for-speed real-time variant of Section 4.2).  The paper
 * names these steps but gives no formulas; every definition below is the
 * reading stated in the design notes, written out directly:
 *
 *   gain selection   low gain iff the highest raw high-gain sample >= switch
 *   window sum       W(s) = sum_{k<w} x[s+k] for every start s in [0, T-w],
 *                    summed directly (no running sum)
 *   window start s*  by the camera's signal extractor (the paper's Section 5
 *                    mentions several extraction algorithms; four are here):
 *                    sliding      first maximiser of W(s) on the pixel's
 *                                 selected gain
 *                    fixed        s0, the same for every pixel; the gain
 *                                 decision looks only at the high-gain
 *                                 samples s0 .. s0+w-1
 *                    global peak  first maximiser of C(s) = the sum over all
 *                                 pixels of the raw high-gain W(s), the same
 *                                 for every pixel of the event
 *                    neighbour    first maximiser of C_i(s) = the sum over
 *                    peak         the pixel's neighbours of their raw
 *                                 high-gain W(s) (0 for a pixel without
 *                                 neighbours, so s* = 0)
 *   pedestal (Q8)    P = nearest-even(256 * ped);  D = 256 * W(s*) - w * P
 *   time numerator   Nt = sum_{k<w} k * (256 * x[s*+k] - P)
 *   charge / time    q = D / (256 * a)  p.e.;  t = s* + Nt / D  (D > 0),
 *                    else s* + (w - 1) / 2
 *   peak index       s* + first argmax of x[s*..s*+w-1]
 *   thresholds       Tx = ceil(256 * a * T_x)  (exact in FP64)
 *   tailcut          mask_i = (D_i >= Tb_i and some neighbour D_j >= Tp_j)
 *                          or (D_i >= Tp_i and some neighbour D_j >= Tb_j)
 *   islands          connected components of the mask (breadth-first search)
 *   Hillas           charge-weighted, centred two-pass moments over the mask
 *   stereo           weighted least-squares intersection of major axes
 *
 * Parity status: every function here is pinned by the CPU-only tests (closed
 * forms, lattice symmetries, brute force, integer identities).  This file
 * shares no code, header or table with the HIP library and includes nothing
 * from it; neighbour lists are derived here from pixel positions by an
 * O(N^2) distance test.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

enum { OR_EX_SLIDING = 0, OR_EX_FIXED = 1, OR_EX_GLOBAL_PEAK = 2, OR_EX_NEIGHBOUR_PEAK = 3 };

typedef struct oracle_cam {
  int32_t n_pix, n_pix_pad, n_samp, n_gain;
  int32_t window, hg_switch, max_nbr, extractor;
  int32_t fixed_start, pad_;
  const float* x;        /* [N] m */
  const float* y;        /* [N] m */
  const float* ped;      /* [G][N] per-sample pedestal, ADC */
  const float* a;        /* [G][N] ADC per p.e. */
  const int32_t* nbr;    /* [N][max_nbr] oracle-built neighbour lists, -1 padded */
  double t_pic, t_bnd;   /* tailcut levels, p.e. */
  double focal;          /* m */
} oracle_cam;

typedef struct oracle_pix {
  int64_t S;       /* raw window sum at s* */
  int64_t D;       /* 256*S - w*P */
  int64_t Nt;      /* time numerator */
  int32_t sstar, peak, gain, pad_;
  double q, t;
} oracle_pix;

typedef struct oracle_hillas {
  double size, cog_x, cog_y, length, width, psi, skewness, kurtosis;
  double time_gradient, time_intercept, leakage, cog_dist;
  int64_t n_pix, n_islands, n_lowgain, flags;
} oracle_hillas;

enum { OR_HILLAS_INVALID = 1, OR_TIME_INVALID = 2, OR_LOW_GAIN = 4 };
enum { OR_STEREO_INVALID = 1 };

/* ------------------------------------------------------------------ */
/* Neighbours by brute force: j != i is a neighbour of i iff           */
/* |r_i - r_j| <= tol.  Lists are ascending in j, -1 padded.           */
/* Returns the largest neighbour count found (or -1 if above max_nbr). */
/* ------------------------------------------------------------------ */
int oracle_neighbours(int32_t n, const float* x, const float* y, double tol, int32_t max_nbr, int32_t* nbr) {
  int32_t most = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t c = 0;
    for (int32_t k = 0; k < max_nbr; ++k) nbr[(int64_t)i * max_nbr + k] = -1;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = (double)x[i] - (double)x[j], dy = (double)y[i] - (double)y[j];
      if (sqrt(dx * dx + dy * dy) <= tol) {
        if (c >= max_nbr) return -1;
        nbr[(int64_t)i * max_nbr + c] = j;
        ++c;
      }
    }
    if (c > most) most = c;
  }
  return most;
}

static int64_t q8_pedestal(float ped) { return (int64_t)nearbyint(256.0 * (double)ped); }

static int64_t q8_threshold(float a, double level) { return (int64_t)ceil(256.0 * (double)a * level); }

/* ------------------------------------------------------------------ */
/* Calibration of one camera event.  ev: uint16 [G][T][Npad].           */
/* ------------------------------------------------------------------ */
void oracle_calibrate_event(const oracle_cam* cam, const uint16_t* ev, oracle_pix* out) {
  const int N = cam->n_pix, Np = cam->n_pix_pad, T = cam->n_samp, G = cam->n_gain, w = cam->window;
  const int ex = cam->extractor, s0 = cam->fixed_start;
  /* global peak: the camera-summed raw high-gain window, first maximiser */
  int sglob = 0;
  if (ex == OR_EX_GLOBAL_PEAK) {
    int64_t cbest = -1;
    for (int s = 0; s + w <= T; ++s) {
      int64_t C = 0;
      for (int j = 0; j < N; ++j)
        for (int k = 0; k < w; ++k) C += ev[(int64_t)(s + k) * Np + j];
      if (C > cbest) { cbest = C; sglob = s; }
    }
  }
  for (int i = 0; i < N; ++i) {
    /* gain selection on the raw high-gain trace (the fixed window looks
       only inside the window) */
    int g = 0;
    if (G == 2) {
      const int k_lo = ex == OR_EX_FIXED ? s0 : 0, k_hi = ex == OR_EX_FIXED ? s0 + w : T;
      int64_t hmax = 0;
      for (int k = k_lo; k < k_hi; ++k) {
        int64_t v = ev[(int64_t)k * Np + i];
        if (v > hmax) hmax = v;
      }
      if (hmax >= cam->hg_switch) g = 1;
    }
    const uint16_t* tr = ev + (int64_t)g * T * Np + i;   /* sample k at tr[k * Np] */
    int64_t best = -1;
    int sbest = 0;
    if (ex == OR_EX_SLIDING) {
      /* every window summed directly; the first maximiser wins */
      for (int s = 0; s + w <= T; ++s) {
        int64_t W = 0;
        for (int k = 0; k < w; ++k) W += tr[(int64_t)(s + k) * Np];
        if (W > best) { best = W; sbest = s; }
      }
    } else {
      if (ex == OR_EX_NEIGHBOUR_PEAK) {
        /* the neighbours' raw high-gain windows, summed directly for every
           start; the first maximiser wins */
        int64_t cbest = -1;
        for (int s = 0; s + w <= T; ++s) {
          int64_t C = 0;
          for (int m = 0; m < cam->max_nbr; ++m) {
            const int j = cam->nbr[(int64_t)i * cam->max_nbr + m];
            if (j < 0) continue;
            for (int k = 0; k < w; ++k) C += ev[(int64_t)(s + k) * Np + j];
          }
          if (C > cbest) { cbest = C; sbest = s; }
        }
      } else {
        sbest = ex == OR_EX_FIXED ? s0 : sglob;
      }
      best = 0;
      for (int k = 0; k < w; ++k) best += tr[(int64_t)(sbest + k) * Np];
    }
    int64_t P = q8_pedestal(cam->ped[g * N + i]);
    int64_t D = 256 * best - (int64_t)w * P;
    int64_t Nt = 0;
    int peak = sbest;
    int64_t pmax = -1;
    for (int k = 0; k < w; ++k) {
      int64_t xv = tr[(int64_t)(sbest + k) * Np];
      Nt += (int64_t)k * (256 * xv - P);
      if (xv > pmax) { pmax = xv; peak = sbest + k; }
    }
    oracle_pix* o = &out[i];
    o->S = best;
    o->D = D;
    o->Nt = Nt;
    o->sstar = sbest;
    o->peak = peak;
    o->gain = g;
    o->q = (double)D / (256.0 * (double)cam->a[g * N + i]);
    o->t = D > 0 ? (double)sbest + (double)Nt / (double)D : (double)sbest + 0.5 * (double)(w - 1);
  }
}

/* ------------------------------------------------------------------ */
/* Two-level tailcut.  D and gain per pixel; mask out [N] (0/1).         */
/* ------------------------------------------------------------------ */
void oracle_clean_event(const oracle_cam* cam, const int64_t* D, const int32_t* gain, uint8_t* mask) {
  const int N = cam->n_pix, M = cam->max_nbr;
  for (int i = 0; i < N; ++i) {
    int gi = gain[i];
    int bnd_i = D[i] >= q8_threshold(cam->a[gi * N + i], cam->t_bnd);
    int pic_i = D[i] >= q8_threshold(cam->a[gi * N + i], cam->t_pic);
    int nb_pic = 0, nb_bnd = 0;
    for (int k = 0; k < M; ++k) {
      int j = cam->nbr[(int64_t)i * M + k];
      if (j < 0) continue;
      int gj = gain[j];
      if (D[j] >= q8_threshold(cam->a[gj * N + j], cam->t_pic)) nb_pic = 1;
      if (D[j] >= q8_threshold(cam->a[gj * N + j], cam->t_bnd)) nb_bnd = 1;
    }
    mask[i] = (uint8_t)((bnd_i && nb_pic) || (pic_i && nb_bnd));
  }
}

/* Connected components of the mask under the neighbour graph (BFS). */
int64_t oracle_islands(const oracle_cam* cam, const uint8_t* mask) {
  const int N = cam->n_pix, M = cam->max_nbr;
  int32_t* seen = (int32_t*)calloc((size_t)N, sizeof(int32_t));
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
  int64_t count = 0;
  for (int i = 0; i < N; ++i) {
    if (!mask[i] || seen[i]) continue;
    ++count;
    int head = 0, tail = 0;
    queue[tail++] = i;
    seen[i] = 1;
    while (head < tail) {
      int u = queue[head++];
      for (int k = 0; k < M; ++k) {
        int v = cam->nbr[(int64_t)u * M + k];
        if (v >= 0 && mask[v] && !seen[v]) { seen[v] = 1; queue[tail++] = v; }
      }
    }
  }
  free(queue);
  free(seen);
  return count;
}

/* ------------------------------------------------------------------ */
/* Hillas parameters over the mask, from q [N] p.e. and t [N] samples.  */
/* ------------------------------------------------------------------ */
void oracle_hillas_event(const oracle_cam* cam, const double* q, const double* t, const uint8_t* mask,
                         const int32_t* gain, oracle_hillas* h) {
  const int N = cam->n_pix, M = cam->max_nbr;
  memset(h, 0, sizeof(*h));
  int64_t n = 0, nlow = 0;
  double S = 0;
  for (int i = 0; i < N; ++i)
    if (mask[i]) { ++n; S += q[i]; }
  for (int i = 0; i < N; ++i)
    if (gain && gain[i] == 1) ++nlow;
  h->n_pix = n;
  h->n_lowgain = nlow;
  h->size = S;
  h->n_islands = oracle_islands(cam, mask);
  if (nlow) h->flags |= OR_LOW_GAIN;
  if (n < 2 || !(S > 0)) {
    h->cog_x = h->cog_y = h->length = h->width = h->psi = NAN;
    h->skewness = h->kurtosis = h->time_gradient = h->time_intercept = NAN;
    h->leakage = h->cog_dist = NAN;
    h->flags |= OR_HILLAS_INVALID | OR_TIME_INVALID;
    return;
  }
  /* first pass: centre of gravity and border (leakage) charge */
  double sx = 0, sy = 0, sborder = 0;
  for (int i = 0; i < N; ++i) {
    if (!mask[i]) continue;
    sx += q[i] * (double)cam->x[i];
    sy += q[i] * (double)cam->y[i];
    int c = 0;
    for (int k = 0; k < M; ++k) c += cam->nbr[(int64_t)i * M + k] >= 0;
    if (c < 6) sborder += q[i];
  }
  double xm = sx / S, ym = sy / S;
  /* second pass: centred second moments */
  double sxx = 0, syy = 0, sxy = 0;
  for (int i = 0; i < N; ++i) {
    if (!mask[i]) continue;
    double dx = (double)cam->x[i] - xm, dy = (double)cam->y[i] - ym;
    sxx += q[i] * dx * dx;
    syy += q[i] * dy * dy;
    sxy += q[i] * dx * dy;
  }
  sxx /= S; syy /= S; sxy /= S;
  double half_diff = 0.5 * (sxx - syy);
  double root = sqrt(half_diff * half_diff + sxy * sxy);
  double lam_p = 0.5 * (sxx + syy) + root;
  double det = sxx * syy - sxy * sxy;
  double lam_m = lam_p > 0 ? det / lam_p : 0.0;
  double psi = 0.5 * atan2(2.0 * sxy, sxx - syy);
  double len = sqrt(lam_p), wid = sqrt(lam_m > 0 ? lam_m : 0.0);
  /* third pass: longitudinal coordinate moments and time-gradient sums */
  double c = cos(psi), s = sin(psi);
  double m3 = 0, m4 = 0, lsum = 0, tsum = 0;
  for (int i = 0; i < N; ++i) {
    if (!mask[i]) continue;
    double l = ((double)cam->x[i] - xm) * c + ((double)cam->y[i] - ym) * s;
    m3 += q[i] * l * l * l;
    m4 += q[i] * l * l * l * l;
    lsum += l;
    tsum += t[i];
  }
  double lbar = lsum / (double)n, tbar = tsum / (double)n;
  double sll = 0, slt = 0;
  for (int i = 0; i < N; ++i) {
    if (!mask[i]) continue;
    double l = ((double)cam->x[i] - xm) * c + ((double)cam->y[i] - ym) * s;
    sll += (l - lbar) * (l - lbar);
    slt += (l - lbar) * (t[i] - tbar);
  }
  h->cog_x = xm;
  h->cog_y = ym;
  h->length = len;
  h->width = wid;
  h->psi = psi;
  h->skewness = m3 / (S * len * len * len);
  h->kurtosis = m4 / (S * len * len * len * len);
  h->leakage = sborder / S;
  h->cog_dist = sqrt(xm * xm + ym * ym);
  if (sll > 0) {
    h->time_gradient = slt / sll;
    h->time_intercept = tbar - h->time_gradient * lbar;
  } else {
    h->time_gradient = h->time_intercept = NAN;
    h->flags |= OR_TIME_INVALID;
  }
}

/* Whole chain for one camera event. */
void oracle_reconstruct_event(const oracle_cam* cam, const uint16_t* ev, oracle_pix* pix, uint8_t* mask,
                              oracle_hillas* h) {
  const int N = cam->n_pix;
  oracle_calibrate_event(cam, ev, pix);
  int64_t* D = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
  int32_t* g = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  double* q = (double*)malloc(sizeof(double) * (size_t)N);
  double* t = (double*)malloc(sizeof(double) * (size_t)N);
  for (int i = 0; i < N; ++i) { D[i] = pix[i].D; g[i] = pix[i].gain; q[i] = pix[i].q; t[i] = pix[i].t; }
  oracle_clean_event(cam, D, g, mask);
  oracle_hillas_event(cam, q, t, mask, g, h);
  free(t); free(q); free(g); free(D);
}

/* ------------------------------------------------------------------ */
/* Stereo direction of one array event.                                 */
/* Minimises sum_i w_i (n_i . (p - c_i))^2 over the nominal-frame point */
/* p, with c_i = cog_i / f_i, n_i = (-sin psi_i, cos psi_i) and         */
/* w_i = size_i (1 - width_i / length_i).  Telescopes with invalid      */
/* Hillas or width/length > 0.9 are dropped; fewer than two telescopes  */
/* or cond(A) >= 1e4 give NaN and the invalid flag.                     */
/* in: [n][5] = size, cog_x, cog_y, length, width; psi [n]; valid [n].  */
/* out: dir_x, dir_y, cond, n_used, flags                               */
/* ------------------------------------------------------------------ */
void oracle_stereo(int32_t n, const double* size, const double* cog_x, const double* cog_y, const double* length,
                   const double* width, const double* psi, const int32_t* valid, const double* focal,
                   double* out) {
  double A00 = 0, A01 = 0, A11 = 0, b0 = 0, b1 = 0;
  int used = 0;
  for (int i = 0; i < n; ++i) {
    if (!valid[i]) continue;
    if (!(length[i] > 0) || !(width[i] >= 0) || !isfinite(psi[i]) || !isfinite(size[i])) continue;
    double ratio = width[i] / length[i];
    if (ratio > 0.9) continue;
    double wgt = size[i] * (1.0 - ratio);
    double nx = -sin(psi[i]), ny = cos(psi[i]);
    double cx = cog_x[i] / focal[i], cy = cog_y[i] / focal[i];
    double nc = nx * cx + ny * cy;
    A00 += wgt * nx * nx;
    A01 += wgt * nx * ny;
    A11 += wgt * ny * ny;
    b0 += wgt * nc * nx;
    b1 += wgt * nc * ny;
    ++used;
  }
  double tr = A00 + A11, det = A00 * A11 - A01 * A01;
  double disc = sqrt(0.25 * (A00 - A11) * (A00 - A11) + A01 * A01);
  double lmax = 0.5 * tr + disc, lmin = 0.5 * tr - disc;
  double cond = (lmin > 0) ? lmax / lmin : INFINITY;
  out[2] = cond;
  out[3] = used;
  if (used < 2 || !(cond < 1e4)) {
    out[0] = out[1] = NAN;
    out[4] = OR_STEREO_INVALID;
    return;
  }
  out[0] = (A11 * b0 - A01 * b1) / det;
  out[1] = (A00 * b1 - A01 * b0) / det;
  out[4] = 0;
}

/* ------------------------------------------------------------------ */
/* Batches: many camera events of several types, optionally threaded.  */
/* ------------------------------------------------------------------ */
typedef struct {
  const oracle_cam* cams;
  const int32_t* types;
  const uint16_t* blob;
  const int64_t* offsets;   /* element offsets of each event's trace block */
  oracle_hillas* out;
  int64_t begin, end;
} batch_job;

static void* batch_worker(void* arg) {
  batch_job* J = (batch_job*)arg;
  int maxN = 0;
  for (int64_t e = J->begin; e < J->end; ++e) {
    int n = J->cams[J->types[e]].n_pix;
    if (n > maxN) maxN = n;
  }
  oracle_pix* pix = (oracle_pix*)malloc(sizeof(oracle_pix) * (size_t)(maxN > 0 ? maxN : 1));
  uint8_t* mask = (uint8_t*)malloc((size_t)(maxN > 0 ? maxN : 1));
  for (int64_t e = J->begin; e < J->end; ++e)
    oracle_reconstruct_event(&J->cams[J->types[e]], J->blob + J->offsets[e], pix, mask, &J->out[e]);
  free(mask);
  free(pix);
  return NULL;
}

void oracle_reconstruct_batch(const oracle_cam* cams, int64_t n_evt, const int32_t* types, const uint16_t* blob,
                              const int64_t* offsets, oracle_hillas* out, int32_t n_threads) {
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  batch_job jobs[256];
  for (int t = 0; t < n_threads; ++t) {
    jobs[t].cams = cams; jobs[t].types = types; jobs[t].blob = blob; jobs[t].offsets = offsets;
    jobs[t].out = out;
    jobs[t].begin = n_evt * t / n_threads;
    jobs[t].end = n_evt * (t + 1) / n_threads;
  }
  for (int t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, batch_worker, &jobs[t]);
  batch_worker(&jobs[0]);
  for (int t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
}

int oracle_sizeof_cam(void) { return (int)sizeof(oracle_cam); }
int oracle_sizeof_pix(void) { return (int)sizeof(oracle_pix); }
int oracle_sizeof_hillas(void) { return (int)sizeof(oracle_hillas); }

/* ------------------------------------------------------------------ */
/* CRC-16 of the DL0 telemetry packets: polynomial x^16+x^12+x^5+1,    */
/* initial register 0xFFFF, bits most-significant first, no final xor, */
/* computed bit by bit from the definition (no table).                 */
/* ------------------------------------------------------------------ */
uint16_t oracle_crc16(const uint8_t* p, int64_t n) {
  uint32_t c = 0xFFFF;
  for (int64_t i = 0; i < n; ++i) {
    c ^= (uint32_t)p[i] << 8;
    for (int b = 0; b < 8; ++b) c = (c & 0x8000) ? ((c << 1) ^ 0x1021) & 0xFFFF : (c << 1) & 0xFFFF;
  }
  return (uint16_t)c;
}
