"""Host check of the batch-descriptor validation (``csrc/descriptors.h``), the
functions the fused reconstruction kernel and the per-array-event kernel call
before they touch a camera event or an array event's telescope range.

A small g++ driver, built with AddressSanitizer and UndefinedBehaviorSanitizer
(no recovery), runs the header's functions on the malformed batch of the GPU
descriptor test (a type index past the table, a misaligned offset, an offset at
the end of the pool, a negative offset, an array event whose range ends before
it starts) and on int64 / int32 extremes, then performs every read the kernels
perform for the accepted descriptors (first and last trace element of each
accepted camera event, each telescope type and record of each accepted array
event) on arrays allocated at their exact sizes, so an accepted descriptor that
reached outside its array, or an overflowing offset sum, aborts the driver.
CPU only."""
import os
import subprocess

import numpy as np
import pytest

import dl0sim

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1307_6489_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")

BAD_TYPE, BAD_OFFSET = 0x1, 0x2
I64_MAX, I64_MIN = 2 ** 63 - 1, -2 ** 63

DRIVER = r"""
#define __host__
#define __device__
#include <cstdio>
#include <cstdint>
#include <vector>
#include "descriptors.h"
// stdin: n_types pool_len elems[n_types] | n_desc (ty off)* | n_tel n_evt offs[n_evt+1] tel_type[n_tel]
int main() {
  int n_types = 0; long long pool_len = 0;
  if (std::scanf("%d %lld", &n_types, &pool_len) != 2) return 2;
  std::vector<long long> elems(n_types);
  for (auto& e : elems) if (std::scanf("%lld", &e) != 1) return 2;
  uint16_t* pool = new uint16_t[pool_len > 0 ? pool_len : 1];
  for (long long i = 0; i < pool_len; ++i) pool[i] = (uint16_t)i;
  int n_desc = 0;
  if (std::scanf("%d", &n_desc) != 1) return 2;
  unsigned long long touched = 0;
  for (int k = 0; k < n_desc; ++k) {
    long long ty = 0, off = 0;
    if (std::scanf("%lld %lld", &ty, &off) != 2) return 2;
    int calls = 0;
    const uint32_t st = rta::tel_descriptor_status((int32_t)ty, (int64_t)off, n_types, pool_len,
                                                   [&](int t) { ++calls; return (int64_t)elems.at(t); });
    if (st == RTA_STATUS_BAD_TYPE && calls != 0) return 4;
    if (st == 0) {  // the kernel's reads of an accepted event
      touched += pool[off] + pool[off + elems[ty] - 1];
    }
    std::printf("T %u\n", st);
  }
  long long n_tel = 0; int n_evt = 0;
  if (std::scanf("%lld %d", &n_tel, &n_evt) != 2) return 2;
  std::vector<long long> eo(n_evt + 1);
  for (auto& v : eo) if (std::scanf("%lld", &v) != 1) return 2;
  int32_t* tel_type = new int32_t[n_tel > 0 ? n_tel : 1];
  float* rec = new float[(n_tel > 0 ? n_tel : 1) * 16];
  for (long long k = 0; k < n_tel; ++k) {
    if (std::scanf("%d", &tel_type[k]) != 1) return 2;
    for (int f = 0; f < 16; ++f) rec[k * 16 + f] = (float)k;
  }
  for (int e = 0; e < n_evt; ++e) {
    const int64_t lo = eo[e], hi = eo[e + 1];
    const bool ok = rta::event_range_ok(lo, hi, n_tel);
    if (ok) {  // the per-event kernel's reads: type and record of each telescope, 16-row tiles
      for (int64_t k = lo; k < hi; ++k) touched += (unsigned)tel_type[k] + (unsigned long long)rec[k * 16 + 15];
      for (int64_t r0 = lo; r0 < hi; r0 += 16)
        for (int col = 0; col < 16; ++col)
          if (r0 + col < hi) touched += (unsigned long long)rec[(r0 + col) * 16];
    }
    std::printf("E %d\n", ok ? 1 : 0);
  }
  std::printf("touched %llu\n", touched);
  delete[] pool;
  delete[] tel_type;
  delete[] rec;
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("descriptors")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC, "-I", INCLUDE, str(src), "-o", str(exe)], check=True)
    return exe


def run(exe, elems, pool_len, desc, n_tel, evt_off, tel_type):
    lines = ["%d %d" % (len(elems), pool_len), " ".join(str(int(e)) for e in elems), str(len(desc))]
    lines += ["%d %d" % (int(t), int(o)) for t, o in desc]
    lines.append("%d %d" % (n_tel, len(evt_off) - 1))
    lines.append(" ".join(str(int(v)) for v in evt_off))
    lines.append(" ".join(str(int(v)) for v in tel_type))
    p = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert p.returncode == 0, p.stderr[-3000:]
    out = p.stdout.split("\n")
    tel = [int(l.split()[1]) for l in out if l.startswith("T ")]
    evt = [int(l.split()[1]) for l in out if l.startswith("E ")]
    return tel, evt


def c1_elems():
    return [c.event_elems for c in dl0sim.camera_types_c1()]


def expected_tel(ty, off, elems, pool_len):
    if not 0 <= ty < len(elems):
        return BAD_TYPE
    n = elems[ty]
    if off < 0 or off % 8 or off + n > pool_len:   # Python integers: no overflow
        return BAD_OFFSET
    return 0


def test_malformed_batch_of_the_gpu_descriptor_test(driver):
    """The eight-telescope batch with a bad type (1), a misaligned offset (3),
    an offset at the pool's end (5) and a negative offset (6), and array
    events [0, 3), [3, 8), [8, 5)."""
    elems = c1_elems()
    ty = np.array([0, 1, 2, 2, 1, 2, 0, 2], np.int64)
    off = np.concatenate([[0], np.cumsum([elems[t] for t in ty])])[:-1].astype(np.int64)
    pool_len = int(sum(elems[t] for t in ty))
    assert all(o % 8 == 0 for o in off)
    ty[1] = 7
    off[3] += 4
    off[5] = pool_len
    off[6] = -8
    tel, evt = run(driver, elems, pool_len, list(zip(ty, off)), 8, [0, 3, 8, 5], ty)
    assert tel == [0, BAD_TYPE, 0, BAD_OFFSET, 0, BAD_OFFSET, BAD_OFFSET, 0]
    assert evt == [1, 1, 0]


def test_offset_and_type_extremes(driver):
    elems = c1_elems()
    pool_len = 3 * max(elems) + 40
    cases = []
    for t in range(3):
        n = elems[t]
        last = (pool_len - n) // 8 * 8          # last aligned start that fits
        cases += [(t, 0), (t, last), (t, last + 8), (t, pool_len - n + 1), (t, pool_len), (t, pool_len + 8),
                  (t, -1), (t, -8), (t, I64_MIN), (t, I64_MAX), (t, I64_MAX - 7), (t, I64_MAX - 15),
                  (t, 8), (t, 4), (t, 2)]
    cases += [(-1, 0), (3, 0), (2 ** 31 - 1, 0), (-2 ** 31, 0), (7, 16)]
    tel, _ = run(driver, elems, pool_len, cases, 0, [0], [])
    assert tel == [expected_tel(t, o, elems, pool_len) for t, o in cases]
    # a pool smaller than one event rejects every offset of that type
    small = elems[0] - 8
    tel, _ = run(driver, elems, small, [(0, 0), (0, 8), (1, 0)], 0, [0], [])
    assert tel == [BAD_OFFSET, BAD_OFFSET, expected_tel(1, 0, elems, small)]


def test_event_range_extremes(driver):
    n_tel = 40
    eo = [0, 0, 17, 40, 39, 41, -1, 5, I64_MAX, I64_MIN, 40, 40, 3]
    _, evt = run(driver, [8], 8, [], n_tel, eo, np.arange(n_tel) % 3)
    exp = [int(0 <= lo <= hi <= n_tel) for lo, hi in zip(eo[:-1], eo[1:])]
    assert evt == exp
    assert evt == [1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 1, 0]
    # no telescopes at all: only empty ranges at 0 are usable
    _, evt = run(driver, [8], 8, [], 0, [0, 0, 1, 0], [])
    assert evt == [1, 0, 0]
