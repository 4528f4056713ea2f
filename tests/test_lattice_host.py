"""Host logic of the lattice-row tables the neighbour-peak stage stages its
words by (``csrc/lattice.h``), compiled with g++ into a small driver: the
order is a permutation, every pixel keeps exactly its neighbour set, a
padding pixel keeps its own slot, and on a hexagonal lattice an interior
pixel's six directions land in the six columns (row before: two adjacent
positions; same row: the positions on either side; row after: two adjacent
positions), so lanes on one row read each direction's words consecutively.
CPU only."""
import os
import subprocess

import numpy as np
import pytest

import dl0sim
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1307_6489_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "lattice.h"
int main(int argc, char** argv) {
  FILE* f = std::fopen(argv[1], "rb");
  int N = 0, Np = 0;
  if (std::fread(&N, 4, 1, f) != 1 || std::fread(&Np, 4, 1, f) != 1) return 2;
  std::vector<float> X(N), Y(N);
  std::vector<int16_t> nb((size_t)N * 8);
  if (std::fread(X.data(), 4, N, f) != (size_t)N || std::fread(Y.data(), 4, N, f) != (size_t)N ||
      std::fread(nb.data(), 2, nb.size(), f) != nb.size()) return 3;
  std::fclose(f);
  std::vector<int16_t> lat((size_t)Np * 8, -1);
  std::vector<uint16_t> lpos(Np, 0);
  rta::lattice_order(N, Np, X.data(), Y.data(), nb.data(), lat.data(), lpos.data());
  FILE* o = std::fopen(argv[2], "wb");
  std::fwrite(lat.data(), 2, lat.size(), o);
  std::fwrite(lpos.data(), 2, lpos.size(), o);
  std::fclose(o);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("lattice")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return d, exe


def tables(driver, x, y, nbr):
    d, exe = driver
    N = len(x)
    Np = (N + 7) // 8 * 8
    nb = -np.ones((N, 8), np.int16)
    nb[:, :nbr.shape[1]] = nbr
    inp, out = d / "in.bin", d / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.array([N, Np], np.int32).tobytes())
        f.write(np.ascontiguousarray(x, np.float32).tobytes())
        f.write(np.ascontiguousarray(y, np.float32).tobytes())
        f.write(nb.tobytes())
    subprocess.run([str(exe), str(inp), str(out)], check=True)
    raw = np.fromfile(out, np.uint16)
    lat = raw[:Np * 8].view(np.int16).reshape(Np, 8)
    lpos = raw[Np * 8:]
    return lat, lpos, Np


def check_consistent(lat, lpos, Np, nbr):
    N = len(nbr)
    order = lat[:N, 6].astype(int)
    assert sorted(order) == list(range(N))                      # a permutation
    assert np.array_equal(lpos[:N][order], np.arange(N))       # lpos inverts it
    assert np.array_equal(lpos[N:], np.arange(N, Np))           # padding keeps its slot
    assert np.all(lat[:N, 7] == -1) and np.all(lat[N:] == -1)
    for p in range(N):
        got = sorted(order[v] for v in lat[p, :6] if v >= 0)
        assert got == sorted(int(j) for j in nbr[order[p]] if j >= 0), p


@pytest.mark.parametrize("n", [7, 61, 1855, 2048])
def test_hexagon_rows(driver, n):
    """The generator's hexagons (pixels in distance order): interior pixels
    get (q, q + 1, p - 1, p + 1, r, r + 1) in the six columns."""
    g = dl0sim.hex_geometry(n)
    lat, lpos, Np = tables(driver, g.x, g.y, g.nbr)
    check_consistent(lat, lpos, Np, g.nbr)
    full = 0
    for p in range(n):
        L = lat[p, :6].astype(int)
        if np.all(L >= 0):
            full += 1
            assert L[2] == p - 1 and L[3] == p + 1, p
            assert L[1] == L[0] + 1 and L[5] == L[4] + 1, p
            assert L[0] < p < L[4], p
    assert full == sum(1 for i in range(n) if np.all(g.nbr[i] >= 0))


def test_other_layouts(driver):
    """A randomly numbered hexagon, a square grid, one row, a jittered
    hexagon and a camera whose positions are all equal apart from x: the
    tables stay a consistent permutation with every neighbour set kept."""
    p = dl0sim.PITCH_M
    rng = np.random.default_rng(31)
    h = dl0sim.hex_geometry(61)
    perm = rng.permutation(61)
    g = np.arange(15) * p
    gx, gy = np.meshgrid(g, g)
    j = dl0sim.hex_geometry(331)
    shapes = [(h.x[perm], h.y[perm]), (gx.ravel(), gy.ravel()), (np.arange(50) * p, np.zeros(50)),
              (j.x + rng.uniform(-0.1, 0.1, 331) * p, j.y + rng.uniform(-0.1, 0.1, 331) * p)]
    for x, y in shapes:
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        nbr = oracle.neighbours(x, y, 1.4 * p)
        lat, lpos, Np = tables(driver, x, y, nbr)
        check_consistent(lat, lpos, Np, nbr)


def test_no_neighbours_and_non_finite_positions(driver):
    """Pixels without neighbours and NaN / infinite positions still give a
    valid permutation (the order only affects speed)."""
    x = np.array([0.0, np.nan, 1.0, np.inf, -np.inf, 2.0, 0.5], np.float32)
    y = np.array([0.0, 0.0, np.nan, 1.0, 0.0, -1.0, 0.5], np.float32)
    nbr = -np.ones((7, 6), np.int32)
    lat, lpos, Np = tables(driver, x, y, nbr)
    check_consistent(lat, lpos, Np, nbr)
