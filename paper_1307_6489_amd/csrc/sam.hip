// HIP kernels of the science alert monitor for gfx950 (CDNA4).
//
// The real-time analysis searches its event list for transients on several
// integration timescales, in a source region and anywhere in the field of
// view (paper, Section 2 requirement (ii); Section 4.2).  The definitions are
// in rta.h.  Three small data-parallel steps:
//   fill     one thread per event: selection, FP64 time bin and sky cell,
//            an integer atomic increment of the counts cube (exact and
//            independent of the order of events);
//   window   one thread per (timescale, 64-bin chunk of the window, cell):
//            the chunk's sum (16 loads in flight, consecutive threads on
//            consecutive cells of a bin) added to the window sum with an
//            integer atomic, so every bin of the longest window is read by
//            its own thread rather than in one long chain;
//   search   one thread per (timescale, cell): on-disc and background-ring
//            sums over a host-built offset list, alpha from the cell counts
//            inside the grid, the Li & Ma significance in FP64 with the zero
//            excess decided in integers, alerts appended through an atomic
//            counter.
#include <algorithm>
#include <cmath>

#include "rta_internal.h"

namespace rta {
namespace {

__global__ void k_sam_clear(int32_t* counts, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    counts[i] = 0;
}

__global__ void k_sam_fill(SamDev d, const rta_event_rec* __restrict__ evt, const double* __restrict__ t,
                           int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const rta_event_rec e = evt[k];
  if (e.flags & RTA_EVT_STEREO_INVALID) return;
  if (!(e.gammaness >= d.gamma_cut)) return;
  const double fb = floor((t[k] - d.t0) / d.bin_s);
  const double half = 0.5 * (double)d.grid;
  const double fx = floor((double)e.dir_x / (double)d.cell + half);
  const double fy = floor((double)e.dir_y / (double)d.cell + half);
  if (!(fb >= 0.0 && fb < (double)d.n_bins && fx >= 0.0 && fx < (double)d.grid && fy >= 0.0 &&
        fy < (double)d.grid))
    return;
  const int64_t G = d.grid;
  atomicAdd(&d.counts[((int64_t)fb * G + (int64_t)fy) * G + (int64_t)fx], 1);
}

// Window jobs of one search: the chunks of timescale s are jobs
// [job0[s], job0[s + 1]), chunk j of it covers bins lo[s] + 64 j .. up to
// end_bin.
constexpr int kSamChunk = 64;
struct SamJobs {
  int32_t job0[RTA_SAM_MAX_SCALES + 1];
  int32_t lo[RTA_SAM_MAX_SCALES];
};

__global__ void k_sam_window(SamDev d, int end_bin, SamJobs jb) {
  const int64_t G2 = (int64_t)d.grid * d.grid;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t job = i / G2;
  if (job >= jb.job0[d.n_scales]) return;
  const int64_t cell = i - job * G2;
  int s = 0;
  while (job >= jb.job0[s + 1]) ++s;
  const int b0 = jb.lo[s] + (int)(job - jb.job0[s]) * kSamChunk;
  const int b1 = min(b0 + kSamChunk, end_bin + 1);
  const int32_t* __restrict__ src = d.counts + cell;
  int32_t acc = 0;
  int b = b0;
  for (; b + 16 <= b1; b += 16) {
    int32_t v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = src[(int64_t)(b + u) * G2];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc += v[u];
  }
  for (; b < b1; ++b) acc += src[(int64_t)b * G2];
  if (acc) atomicAdd(&d.win[s * G2 + cell], acc);
}

__device__ double li_ma(int64_t n_on, int64_t n_off, int64_t c_on, int64_t c_off) {
  if (c_off <= 0 || n_on * c_off == c_on * n_off) return 0.0;
  const double on = (double)n_on, off = (double)n_off, alpha = (double)c_on / (double)c_off;
  const double tot = on + off;
  const double t1 = n_on > 0 ? on * log((1.0 + alpha) / alpha * on / tot) : 0.0;
  const double t2 = n_off > 0 ? off * log((1.0 + alpha) * off / tot) : 0.0;
  const double v = fmax(2.0 * (t1 + t2), 0.0);
  return copysign(sqrt(v), on - alpha * off);
}

__global__ void k_sam_search(SamDev d, double* __restrict__ sig, int32_t* __restrict__ non_out,
                             int32_t* __restrict__ noff_out, rta_sam_alert* __restrict__ alerts, int max_alerts,
                             int32_t* n_alerts) {
  const int G = d.grid;
  const int64_t G2 = (int64_t)G * G;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G2 * d.n_scales) return;
  const int s = (int)(i / G2);
  const int cell = (int)(i - s * G2);
  const int y = cell / G, x = cell - y * G;
  const int32_t* W = d.win + s * G2;
  // branch-free body (cells outside the grid read a clamped cell and add
  // nothing), unrolled so that several window-sum loads are in flight
  int64_t n_on = 0, n_off = 0, c_on = 0, c_off = 0;
#pragma unroll 8
  for (int k = 0; k < d.n_offs; ++k) {
    const int32_t o = d.offs[k];
    const int xx = x + (o & 0xFF) - 128, yy = y + ((o >> 8) & 0xFF) - 128;
    const bool in = xx >= 0 && xx < G && yy >= 0 && yy < G;
    const int32_t v = W[(int64_t)min(max(yy, 0), G - 1) * G + min(max(xx, 0), G - 1)];
    const int64_t vi = in ? (int64_t)v : 0;
    const int64_t ci = in ? 1 : 0;
    const bool on = (o >> 16) == 1;
    n_on += on ? vi : 0;
    c_on += on ? ci : 0;
    n_off += on ? 0 : vi;
    c_off += on ? 0 : ci;
  }
  const double S = li_ma(n_on, n_off, c_on, c_off);
  if (sig) sig[i] = S;
  if (non_out) non_out[i] = (int32_t)n_on;
  if (noff_out) noff_out[i] = (int32_t)n_off;
  if (S >= (double)d.sigma_alert) {
    const int slot = atomicAdd(n_alerts, 1);
    if (slot < max_alerts) {
      rta_sam_alert a;
      a.scale = s;
      a.ix = x;
      a.iy = y;
      a.n_on = (int32_t)n_on;
      a.significance = S;
      a.n_off = (int32_t)n_off;
      a.pad_ = 0;
      alerts[slot] = a;
    }
  }
}

__global__ void k_zero_i32(int32_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

unsigned blocks_for(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

}  // namespace

hipError_t launch_sam_clear(const SamDev& d, hipStream_t st) {
  const int64_t n = (int64_t)d.n_bins * d.grid * d.grid;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_sam_clear, dim3((unsigned)blocks), dim3(256), 0, st, d.counts, n);
  return hipGetLastError();
}

hipError_t launch_sam_fill(const SamDev& d, const rta_event_rec* evt, const double* t, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_sam_fill, dim3(blocks_for(n, 256)), dim3(256), 0, st, d, evt, t, n);
  return hipGetLastError();
}

hipError_t launch_sam_search(const SamDev& d, int end_bin, double* sig, int32_t* n_on, int32_t* n_off,
                             rta_sam_alert* alerts, int max_alerts, int32_t* n_alerts, hipStream_t st) {
  const int64_t G2 = (int64_t)d.grid * d.grid, n = (int64_t)d.n_scales * G2;
  SamJobs jb;
  jb.job0[0] = 0;
  for (int s = 0; s < d.n_scales; ++s) {
    jb.lo[s] = std::max(end_bin - d.scales[s] + 1, 0);
    jb.job0[s + 1] = jb.job0[s] + (end_bin - jb.lo[s] + kSamChunk) / kSamChunk;
  }
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, n_alerts);
  hipLaunchKernelGGL(k_sam_clear, dim3(blocks_for(n, 256)), dim3(256), 0, st, d.win, n);
  hipLaunchKernelGGL(k_sam_window, dim3(blocks_for(jb.job0[d.n_scales] * G2, 256)), dim3(256), 0, st, d, end_bin,
                     jb);
  hipLaunchKernelGGL(k_sam_search, dim3(blocks_for(n, 256)), dim3(256), 0, st, d, sig, n_on, n_off, alerts,
                     max_alerts, n_alerts);
  return hipGetLastError();
}

}  // namespace rta
