// HIP kernels of the real-time health monitor for gfx950 (CDNA4).
//
// A basic quality check of the acquired data (paper, Section 4.2): per pixel
// and gain, the sample count, sum, sum of squares and saturated samples over
// a batch of camera events of one type, then mean / rms, the camera's median
// rms and the bad-pixel flags (definitions in rta.h).
//   accumulate  workgroups take events in turn; each lane owns 8
//               consecutive pixels and streams their 16-byte slices
//               (non-temporal loads: the traces are read once), keeping
//               64-bit sums in registers across its events, and stores them
//               to its workgroup's partial block at the end;
//   reduce      per pixel and quantity, the sum of the partial blocks (16
//               slices of blocks per output, combined in LDS), so the totals
//               are exact integers independent of the schedule;
//   evaluate    one workgroup per gain: FP64 mean / rms without
//               contraction, a bitonic sort of the rms (registers, lane
//               shuffles and LDS) for the lower median, the flags;
//   verdict     one workgroup: pixels flagged in any gain, the verdict.
#include <cmath>

#include "rta_internal.h"

namespace rta {
namespace {

constexpr int kHealthNT = 256;
constexpr int kHealthPPL = 8;
constexpr int kEvalNT = 1024;
constexpr int kWave = 64;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// part: [gridDim.x][3][G][Npad] = s1, s2, n_sat of this workgroup's events
__global__ __launch_bounds__(kHealthNT) void k_health_accum(DevCam c, const uint16_t* __restrict__ traces,
                                                            int64_t n_evt, uint64_t* __restrict__ part) {
  const int N = c.n_pix, np = c.n_pix_pad, T = c.n_samp, G = c.n_gain;
  const int pix0 = (int)threadIdx.x * kHealthPPL;
  const bool act = pix0 < np;
  const uint32_t lvl0 = G == 2 ? (uint32_t)c.hg_switch : 65535u;
  uint64_t s1[2][kHealthPPL], s2[2][kHealthPPL];
  uint32_t ns[2][kHealthPPL];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int p = 0; p < kHealthPPL; ++p) { s1[g][p] = 0; s2[g][p] = 0; ns[g][p] = 0; }
  if (act) {
    for (int64_t e = blockIdx.x; e < n_evt; e += gridDim.x) {
      const uint16_t* ev = traces + e * c.event_elems;
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        if (g >= G) break;
        const uint32_t lvl = g == 0 ? lvl0 : 65535u;
        uint32_t e1[kHealthPPL];
#pragma unroll
        for (int p = 0; p < kHealthPPL; ++p) e1[p] = 0;
        const uint16_t* col = ev + (size_t)g * T * np + pix0;
        // slices in groups of eight, double buffered: the next group's loads
        // are in flight while the current group is reduced (slots past T
        // re-read the last slice and are not accumulated)
        auto load8 = [&](u32x4 (&d)[8], int k0) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int k = min(k0 + j, T - 1);
            d[j] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(col + (size_t)k * np));
          }
        };
        auto take8 = [&](const u32x4 (&d)[8], int k0) {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            if (k0 + j >= T) continue;
#pragma unroll
            for (int p = 0; p < kHealthPPL; ++p) {
              const uint32_t x = (d[j][p >> 1] >> ((p & 1) * 16)) & 0xFFFFu;
              e1[p] += x;
              s2[g][p] += (uint64_t)(x * x);
              ns[g][p] += x >= lvl ? 1u : 0u;
            }
          }
        };
        u32x4 A[8], B[8];
        load8(A, 0);
        for (int k0 = 0; k0 < T; k0 += 16) {
          if (k0 + 8 < T) load8(B, k0 + 8);
          take8(A, k0);
          if (k0 + 8 >= T) break;
          if (k0 + 16 < T) load8(A, k0 + 16);
          take8(B, k0 + 8);
        }
#pragma unroll
        for (int p = 0; p < kHealthPPL; ++p) s1[g][p] += e1[p];
      }
    }
  }
  if (!act) return;
  // padding pixels (i >= N) store zeros
  const int64_t plane = (int64_t)G * np;
  uint64_t* __restrict__ dst = part + (int64_t)blockIdx.x * 3 * plane;
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    if (g >= G) break;
#pragma unroll
    for (int p = 0; p < kHealthPPL; ++p) {
      const int i = pix0 + p;
      const bool real = i < N;
      const int64_t o = (int64_t)g * np + i;
      dst[o] = real ? s1[g][p] : 0ull;
      dst[plane + o] = real ? s2[g][p] : 0ull;
      dst[2 * plane + o] = real ? (uint64_t)ns[g][p] : 0ull;
    }
  }
}

// acc[o] = sum over the n_part partial blocks of part[w][o], o < n_out.  A
// workgroup owns 16 consecutive outputs; its 16 lane groups sum every 16th
// block (16 loads in flight per lane), then LDS adds the 16 group sums.
constexpr int kRedOut = 16, kRedSlices = 16;

__global__ __launch_bounds__(kRedOut * kRedSlices) void k_health_reduce(const uint64_t* __restrict__ part,
                                                                        int64_t n_out, int n_part,
                                                                        uint64_t* __restrict__ acc) {
  __shared__ uint64_t red[kRedSlices][kRedOut];
  const int ol = threadIdx.x % kRedOut, sl = threadIdx.x / kRedOut;
  const int64_t o = (int64_t)blockIdx.x * kRedOut + ol;
  uint64_t s = 0;
  if (o < n_out) {
    int w = sl;
    for (; w + kRedSlices * 15 < n_part; w += kRedSlices * 16) {
      uint64_t v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = part[(int64_t)(w + kRedSlices * u) * n_out + o];
#pragma unroll
      for (int u = 0; u < 16; ++u) s += v[u];
    }
    for (; w < n_part; w += kRedSlices) s += part[(int64_t)w * n_out + o];
  }
  red[sl][ol] = s;
  __syncthreads();
  if (threadIdx.x < kRedOut && o < n_out) {
    uint64_t t = 0;
#pragma unroll
    for (int k = 0; k < kRedSlices; ++k) t += red[k][threadIdx.x];
    acc[o] = t;
  }
}

__device__ __forceinline__ void pixel_stats(uint64_t s1, uint64_t s2, uint64_t n, double& mean, double& rms) {
#pragma clang fp contract(off)
  const double dn = (double)n;
  mean = (double)s1 / dn;
  const double var = (double)s2 / dn - mean * mean;
  rms = sqrt(var > 0.0 ? var : 0.0);
}

// One compare-exchange step of a bitonic sort (ascending overall) for the
// element at index i against its partner's value p: i ^ j is the partner,
// (i & k) the direction of the block being merged.
__device__ __forceinline__ double bitonic_step(double v, double p, int i, int j, int k) {
  const bool take_min = ((i & j) == 0) == ((i & k) == 0);
  return take_min ? fmin(v, p) : fmax(v, p);
}

// Evaluation, one workgroup per gain: thread t owns pixels t and t + 1024.
// The gain's rms, padded with +inf to 2048 values, is sorted ascending by a
// bitonic network on registers: partners within a wavefront (j < 64) by
// lane shuffles, across wavefronts through LDS, j = 1024 inside the thread.
static_assert(2 * kEvalNT == kMaxPix, "two pixels per evaluation thread");

__global__ __launch_bounds__(kEvalNT) void k_health_eval(DevCam c, const uint64_t* __restrict__ acc, int64_t n_evt,
                                                         rta_health_params prm, rta_pixel_health* __restrict__ pix,
                                                         rta_camera_health* __restrict__ out) {
  __shared__ double xch[kMaxPix];
  __shared__ double s_med;
  const int N = c.n_pix, np = c.n_pix_pad, G = c.n_gain;
  const int g = blockIdx.x, t = threadIdx.x;
  const uint64_t n = (uint64_t)n_evt * (uint64_t)c.n_samp;
  const int64_t plane = (int64_t)G * np;
  uint64_t a1[2], a2[2], a3[2];
  double mean[2], rms[2], v[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int i = t + kEvalNT * e;
    a1[e] = a2[e] = a3[e] = 0;
    mean[e] = rms[e] = 0.0;
    v[e] = INFINITY;
    if (i < N) {
      const int64_t o = (int64_t)g * np + i;
      a1[e] = acc[o];
      a2[e] = acc[plane + o];
      a3[e] = acc[2 * plane + o];
      pixel_stats(a1[e], a2[e], n, mean[e], rms[e]);
      v[e] = rms[e];
    }
  }
#pragma unroll
  for (int k = 2; k <= kMaxPix; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      double p[2];
      if (j == kEvalNT) {
        p[0] = v[1];
        p[1] = v[0];
      } else if (j >= kWave) {
        xch[t] = v[0];
        xch[t + kEvalNT] = v[1];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 2; ++e) p[e] = xch[(t + kEvalNT * e) ^ j];
        __syncthreads();
      } else {
#pragma unroll
        for (int e = 0; e < 2; ++e) p[e] = __shfl_xor(v[e], j, kWave);
      }
#pragma unroll
      for (int e = 0; e < 2; ++e) v[e] = bitonic_step(v[e], p[e], t + kEvalNT * e, j, k);
    }
  }
  // lower median: sorted element (N - 1) / 2
  const int mi = (N - 1) / 2;
#pragma unroll
  for (int e = 0; e < 2; ++e)
    if (t + kEvalNT * e == mi) {
      s_med = v[e];
      out->median_rms[g] = v[e];
    }
  __syncthreads();
  const double med = s_med;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int i = t + kEvalNT * e;
    if (i >= N) continue;
    uint32_t f = 0;
    if (rms[e] < (double)prm.rms_dead) f |= RTA_HEALTH_DEAD;
    if (rms[e] > (double)prm.noisy_factor * med) f |= RTA_HEALTH_NOISY;
    const double ped = (double)c.P256[g * np + i] / 256.0;
    if (fabs(mean[e] - ped) > (double)prm.ped_tol) f |= RTA_HEALTH_PED_SHIFT;
    if ((double)a3[e] > (double)prm.sat_frac * (double)n) f |= RTA_HEALTH_SATURATING;
    rta_pixel_health h;
    h.n = n;
    h.s1 = a1[e];
    h.s2 = a2[e];
    h.n_sat = a3[e];
    h.mean = mean[e];
    h.rms = rms[e];
    h.flags = f;
    h.pad_ = 0;
    h.reserved_ = 0;
    pix[(int64_t)g * N + i] = h;
  }
}

// Verdict: pixels with a flag in any gain, from the records just written.
__global__ __launch_bounds__(kEvalNT) void k_health_verdict(DevCam c, rta_health_params prm,
                                                            const rta_pixel_health* __restrict__ pix,
                                                            rta_camera_health* __restrict__ out) {
  __shared__ int32_t nbad;
  const int N = c.n_pix, G = c.n_gain;
  if (threadIdx.x == 0) nbad = 0;
  __syncthreads();
  int mine = 0;
  for (int i = threadIdx.x; i < N; i += kEvalNT) {
    uint32_t any = pix[i].flags;
    if (G == 2) any |= pix[(int64_t)N + i].flags;
    mine += any ? 1 : 0;
  }
  if (mine) atomicAdd(&nbad, mine);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (G == 1) out->median_rms[1] = 0.0;
    out->n_bad = nbad;
    out->verdict = (double)nbad > (double)prm.bad_frac_max * (double)N ? 1 : 0;
  }
}

}  // namespace

hipError_t launch_health(const DevCam& c, const uint16_t* traces, int64_t n_evt, const rta_health_params& p,
                         uint64_t* part, uint64_t* acc, rta_pixel_health* pix, rta_camera_health* out,
                         hipStream_t st) {
  const int64_t n_out = (int64_t)3 * c.n_gain * c.n_pix_pad;
  // each workgroup takes several events; two workgroups per compute unit
  // keep enough loads in flight
  const int grid = (int)(n_evt < kHealthParts ? n_evt : kHealthParts);
  hipLaunchKernelGGL(k_health_accum, dim3((unsigned)grid), dim3(kHealthNT), 0, st, c, traces, n_evt, part);
  hipLaunchKernelGGL(k_health_reduce, dim3((unsigned)((n_out + kRedOut - 1) / kRedOut)), dim3(kRedOut * kRedSlices),
                     0, st, (const uint64_t*)part, n_out, grid, acc);
  hipLaunchKernelGGL(k_health_eval, dim3((unsigned)c.n_gain), dim3(kEvalNT), 0, st, c, (const uint64_t*)acc, n_evt, p,
                     pix, out);
  hipLaunchKernelGGL(k_health_verdict, dim3(1), dim3(kEvalNT), 0, st, c, p, (const rta_pixel_health*)pix, out);
  return hipGetLastError();
}

}  // namespace rta
