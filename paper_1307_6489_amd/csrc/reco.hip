// HIP kernels of the low-level reconstruction for gfx950 (CDNA4).
//
// Calibration / signal extraction, two-level tailcut cleaning, islands and
// Hillas moments of camera events (the calibration and image-parameter stage
// of the real-time reconstruction, Sections 4.1-4.2 of the paper), plus the
// per-array-event stereo direction.  The operations are defined in rta.h.
//
// Data flow of one camera event inside a workgroup:
//   1. extraction   each lane owns PPL consecutive pixels and streams their
//                   samples slice by slice (one PPL*2-byte load per slice, a
//                   wavefront reads 64*PPL*2 contiguous bytes).  A running
//                   w-sample window sum lives in registers; the argmax is a
//                   single unsigned max of (W << 8 | 255 - s).  Dual-gain
//                   cameras track the raw high-gain maximum with packed
//                   16-bit max and re-stream the low gain only for lanes that
//                   own a switched pixel.  D and the threshold flags go to LDS.
//   2. mask         neighbour flags gathered from LDS, one ballot per
//                   64-pixel word.
//   3. compaction   popcount prefix over the mask words gives every cleaned
//                   pixel a slot; q, x, y and the peak time (window samples
//                   re-read for cleaned pixels only) are stored per slot.
//   4. islands      lock-free union-find over the slots in LDS.
//   5. Hillas       four block reductions (cog, centred second moments,
//                   longitudinal moments + time sums, time-gradient sums),
//                   each a fixed-order wavefront butterfly + wave-ordered sum,
//                   so results are deterministic.
#include <cfloat>
#include <cmath>

#include "descriptors.h"
#include "mlp_device.h"
#include "rta_internal.h"

namespace rta {
namespace {

constexpr int kWave = 64;
constexpr float kNaN = __builtin_nanf("");

__device__ __forceinline__ uint32_t lo16(uint32_t d) { return d & 0xffffu; }
__device__ __forceinline__ uint32_t hi16(uint32_t d) { return d >> 16; }

typedef unsigned short us2 __attribute__((ext_vector_type(2)));

// Per-halfword unsigned maximum of two packed pairs of uint16.
__device__ __forceinline__ uint32_t pkmax16(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t,
                            __builtin_elementwise_max(__builtin_bit_cast(us2, a), __builtin_bit_cast(us2, b)));
}

// Trace loads go through a buffer resource spanning one camera event: the
// per-lane byte offset (its pixel group) stays in one VGPR and the per-slice
// offset is wave-uniform, so it rides in the scalar soffset operand.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Cache-policy bits of the trace loads (bit 1 = non-temporal: every trace
// byte is read once, so the L2 should not keep it).
#ifndef RTA_TRACE_CPOL
#define RTA_TRACE_CPOL 2
#endif

__device__ __forceinline__ __amdgpu_buffer_rsrc_t event_rsrc(const uint16_t* base, int64_t elems) {
  // word 3 = 0x00020000: raw 32-bit data format, bounds-checked against num_records
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(base), 0, (int)(elems * 2), 0x00020000);
}

template <int ND>
__device__ __forceinline__ void load_slice(uint32_t (&d)[ND], __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (ND == 4) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, RTA_TRACE_CPOL);
    d[0] = v[0]; d[1] = v[1]; d[2] = v[2]; d[3] = v[3];
  } else if constexpr (ND == 2) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, RTA_TRACE_CPOL);
    d[0] = v[0]; d[1] = v[1];
  } else {
    d[0] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, RTA_TRACE_CPOL);
  }
}

template <int PPL>
__device__ __forceinline__ void load_i32(int32_t (&v)[PPL], const int32_t* p) {
  if constexpr (PPL == 8) {
    const int4 a = *reinterpret_cast<const int4*>(p);
    const int4 b = *reinterpret_cast<const int4*>(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else if constexpr (PPL == 4) {
    const int4 a = *reinterpret_cast<const int4*>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  } else {
    const int2 a = *reinterpret_cast<const int2*>(p);
    v[0] = a.x; v[1] = a.y;
  }
}

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uniform_i64(long long v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(unsigned long long)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  return reinterpret_cast<T*>(uniform_i64(reinterpret_cast<long long>(p)));
}

// A wave-uniform copy of a camera's tables: every field forced into scalar
// registers, so loops over samples / pixels and buffer descriptors built from
// them stay scalar (no per-lane waterfall around buffer loads).
__device__ __forceinline__ DevCam uniform_cam(const DevCam& c) {
  DevCam u;
  u.n_pix = uniform_i32(c.n_pix);
  u.n_pix_pad = uniform_i32(c.n_pix_pad);
  u.n_samp = uniform_i32(c.n_samp);
  u.n_gain = uniform_i32(c.n_gain);
  u.window = uniform_i32(c.window);
  u.hg_switch = uniform_i32(c.hg_switch);
  u.event_elems = uniform_i64(c.event_elems);
  u.focal = __int_as_float(uniform_i32(__float_as_int(c.focal)));
  u.fixed_start = uniform_i32(c.fixed_start);
  u.P256 = uniform_ptr(c.P256);
  u.thr_pic = uniform_ptr(c.thr_pic);
  u.thr_bnd = uniform_ptr(c.thr_bnd);
  u.a = uniform_ptr(c.a);
  u.x = uniform_ptr(c.x);
  u.y = uniform_ptr(c.y);
  u.nbr = uniform_ptr(c.nbr);
  u.border = uniform_ptr(c.border);
  u.crc_tab = uniform_ptr(c.crc_tab);
  return u;
}

// ---------------------------------------------------------------------------
// Sliding-window argmax over one pixel group.
// p0 points at sample 0 of the group's first pixel; sample k of the group is
// the PPL*2 bytes at p0 + k*np.  On return key[p] = max over starts s of
// (W(s) << 8) | (255 - s): the largest window sum, ties to the smallest s.
// With TRACK_MAX, rmax holds the packed per-pixel raw maximum over all T.
//
// Samples stream in chunks of CH slices, double buffered: the loads of chunk
// c+1 are in flight while chunk c is reduced, so a wavefront keeps up to 2*CH
// slice loads outstanding.  Slices past the end of the trace (the tail of the
// last chunk) read whatever follows in the event, or 0 beyond the buffer's
// bounds, and are ignored by the uniform k < T guard.
// ---------------------------------------------------------------------------
template <int PPL, int CH>
__device__ __forceinline__ void load_chunk(uint32_t (&buf)[CH][PPL / 2], __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                           uint32_t sbase, uint32_t stride, int k0) {
  uint32_t soff = sbase + (uint32_t)k0 * stride;
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    load_slice<PPL / 2>(buf[j], r, voff, soff);
    soff += stride;
  }
}

// Slice j of the chunk starting at k0 enters the window whose start is
// k0 + j - W + 1; the sample leaving it is slice j - W of the same chunk, or
// slice CH + j - W of the previous chunk (still intact: the next prefetch into
// that buffer is issued only after the first W slices are reduced).
//
// Within a chunk the candidates are ranked by a chunk-local key
// (W << 4) | (15 - j): the largest sum, then the earliest slice, with an
// inline-constant low part.  merge_chunk folds the chunk's best into the
// global key (W << 8) | (255 - s).
template <int PPL, int W, int CH, bool TRACK_MAX, bool GUARD, bool FIRST, int J0, int J1>
__device__ __forceinline__ void reduce_slices(const uint32_t (&cur)[CH][PPL / 2], const uint32_t (&prev)[CH][PPL / 2],
                                              int k0, int T, uint32_t (&ws)[PPL], uint32_t (&loc)[PPL],
                                              uint32_t (&rmax)[PPL / 2]) {
  constexpr int ND = PPL / 2;
#pragma unroll
  for (int j = J0; j < J1; ++j) {
    if (GUARD && k0 + j >= T) continue;
#pragma unroll
    for (int h = 0; h < ND; ++h) {
      const uint32_t nw = cur[j][h];
      if constexpr (TRACK_MAX) rmax[h] = pkmax16(rmax[h], nw);
      if (FIRST && j < W) {
        ws[2 * h] += lo16(nw);
        ws[2 * h + 1] += hi16(nw);
        if (j == W - 1) {
          loc[2 * h] = max(loc[2 * h], (ws[2 * h] << 4) | (uint32_t)(15 - j));
          loc[2 * h + 1] = max(loc[2 * h + 1], (ws[2 * h + 1] << 4) | (uint32_t)(15 - j));
        }
      } else {
        const uint32_t od = (j >= W) ? cur[j - W][h] : prev[CH + j - W][h];
        ws[2 * h] += lo16(nw) - lo16(od);
        ws[2 * h + 1] += hi16(nw) - hi16(od);
        loc[2 * h] = max(loc[2 * h], (ws[2 * h] << 4) | (uint32_t)(15 - j));
        loc[2 * h + 1] = max(loc[2 * h + 1], (ws[2 * h + 1] << 4) | (uint32_t)(15 - j));
      }
    }
  }
}

// Global key from the chunk-local best: start s = k0 + j - W + 1, so
// 255 - s = (254 - k0 + W - 15) + (15 - j).
template <int PPL, int W>
__device__ __forceinline__ void merge_chunk(int k0, uint32_t (&loc)[PPL], uint32_t (&key)[PPL]) {
  const uint32_t c = (uint32_t)(254 - k0 + W - 15);
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    const uint32_t cand = ((loc[p] >> 4) << 8) | (c + (loc[p] & 15u));
    key[p] = max(key[p], cand);
    loc[p] = 0;
  }
}

template <int PPL, int W, int CH, bool TRACK_MAX, bool GUARD, bool FIRST>
__device__ __forceinline__ void reduce_chunk(const uint32_t (&cur)[CH][PPL / 2], const uint32_t (&prev)[CH][PPL / 2],
                                             int k0, int T, uint32_t (&ws)[PPL], uint32_t (&loc)[PPL],
                                             uint32_t (&key)[PPL], uint32_t (&rmax)[PPL / 2]) {
  reduce_slices<PPL, W, CH, TRACK_MAX, GUARD, FIRST, 0, CH>(cur, prev, k0, T, ws, loc, rmax);
  merge_chunk<PPL, W>(k0, loc, key);
}

template <int PPL, int W, int CH, bool TRACK_MAX>
__device__ __forceinline__ void window_argmax(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t sbase, uint32_t stride,
                                              int T, uint32_t (&key)[PPL], uint32_t (&rmax)[PPL / 2]) {
  static_assert(CH % W == 0 && CH >= W && CH <= 16, "chunk must be a multiple of the window, at most 16");
  constexpr int ND = PPL / 2;
  uint32_t ws[PPL], loc[PPL];
  uint32_t A[CH][ND], B[CH][ND];
#pragma unroll
  for (int p = 0; p < PPL; ++p) { ws[p] = 0; loc[p] = 0; key[p] = 0; }
  const int nchunk = (T + CH - 1) / CH;
  const int nfull = T / CH;  // chunks with all CH slices inside the trace
  load_chunk<PPL, CH>(A, r, voff, sbase, stride, 0);
  if (nchunk > 1) load_chunk<PPL, CH>(B, r, voff, sbase, stride, CH);
  if (nfull >= 1)
    reduce_chunk<PPL, W, CH, TRACK_MAX, false, true>(A, A, 0, T, ws, loc, key, rmax);
  else
    reduce_chunk<PPL, W, CH, TRACK_MAX, true, true>(A, A, 0, T, ws, loc, key, rmax);
  // Chunk c lives in B (odd c) or A (even c); the other buffer holds c - 1.
  for (int c = 1; c < nchunk; c += 2) {
    const int k0 = c * CH;
    if (c < nfull) {
      reduce_slices<PPL, W, CH, TRACK_MAX, false, false, 0, W>(B, A, k0, T, ws, loc, rmax);
      if (c + 1 < nchunk) load_chunk<PPL, CH>(A, r, voff, sbase, stride, k0 + CH);
      reduce_slices<PPL, W, CH, TRACK_MAX, false, false, W, CH>(B, A, k0, T, ws, loc, rmax);
    } else {
      reduce_slices<PPL, W, CH, TRACK_MAX, true, false, 0, CH>(B, A, k0, T, ws, loc, rmax);
    }
    merge_chunk<PPL, W>(k0, loc, key);
    if (c + 1 >= nchunk) break;
    const int k1 = k0 + CH;
    if (c + 1 < nfull) {
      reduce_slices<PPL, W, CH, TRACK_MAX, false, false, 0, W>(A, B, k1, T, ws, loc, rmax);
      if (c + 2 < nchunk) load_chunk<PPL, CH>(B, r, voff, sbase, stride, k1 + CH);
      reduce_slices<PPL, W, CH, TRACK_MAX, false, false, W, CH>(A, B, k1, T, ws, loc, rmax);
    } else {
      reduce_slices<PPL, W, CH, TRACK_MAX, true, false, 0, CH>(A, B, k1, T, ws, loc, rmax);
    }
    merge_chunk<PPL, W>(k1, loc, key);
  }
}

// Extraction of one pixel group on its selected gain.  Returns the bit mask
// of pixels that switched to low gain.
template <int PPL, int W, int CH>
__device__ __forceinline__ uint32_t extract_group(const DevCam& c, __amdgpu_buffer_rsrc_t r, int pix0, int np, int T,
                                                  bool dual, uint32_t (&key)[PPL]) {
  uint32_t rmax[PPL / 2];
#pragma unroll
  for (int h = 0; h < PPL / 2; ++h) rmax[h] = 0;
  const uint32_t voff = (uint32_t)pix0 * 2u, stride = (uint32_t)np * 2u;
  uint32_t sw = 0;
  if (dual) {
    window_argmax<PPL, W, CH, true>(r, voff, 0u, stride, T, key, rmax);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const uint32_t m = (p & 1) ? hi16(rmax[p >> 1]) : lo16(rmax[p >> 1]);
      if ((int)m >= c.hg_switch) sw |= 1u << p;
    }
    // re-stream the low gain when any lane of the wave owns a switched pixel
    // (a wave-uniform branch keeps the buffer operands scalar)
    if (__ballot(sw != 0u)) {
      uint32_t kl[PPL], unused[PPL / 2];
      window_argmax<PPL, W, CH, false>(r, voff, (uint32_t)T * stride, stride, T, kl, unused);
#pragma unroll
      for (int p = 0; p < PPL; ++p)
        if ((sw >> p) & 1u) key[p] = kl[p];
    }
  } else {
    window_argmax<PPL, W, CH, false>(r, voff, 0u, stride, T, key, rmax);
  }
  return sw;
}

// ---------------------------------------------------------------------------
// Sliding-window argmax that also keeps each pixel's best window (the
// unfused calibration call reports Nt and the peak of every pixel, not only of
// the cleaned ones, so re-reading the window samples afterwards would fetch
// scattered rows of the whole trace a second time).  While the samples
// stream past, the window ending at slice k replaces the best one when its
// sum is strictly larger (ties keep the earliest start, as the packed key
// does), and then the window's four samples, already in registers, are kept
// packed two per register.  W = 4 only.
// ---------------------------------------------------------------------------
template <int PPL>
struct KeepState {
  uint32_t ws[PPL];   // running window sum
  uint32_t key[PPL];  // best (sum << 8) | (255 - start) so far (0 before the first window)
  uint32_t sv0[PPL];  // samples s*, s*+1 of the best window (low, high half)
  uint32_t sv1[PPL];  // samples s*+2, s*+3
};

// (half of word a, the same half of word b) packed low / high: the samples
// of one pixel at two consecutive slices.
template <int HALF>
__device__ __forceinline__ uint32_t pair16(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_perm(b, a, HALF ? 0x07060302u : 0x05040100u);
}

template <int PPL, int CH, bool TRACK_MAX, bool GUARD, bool FIRST, int J0, int J1>
__device__ __forceinline__ void keep_slices(const uint32_t (&cur)[CH][PPL / 2], const uint32_t (&prev)[CH][PPL / 2],
                                            int k0, int T, KeepState<PPL>& st, uint32_t (&rmax)[PPL / 2]) {
  constexpr int ND = PPL / 2, W = 4;
#pragma unroll
  for (int j = J0; j < J1; ++j) {
    if (GUARD && k0 + j >= T) continue;
#pragma unroll
    for (int h = 0; h < ND; ++h) {
      const uint32_t nw = cur[j][h];
      if constexpr (TRACK_MAX) rmax[h] = pkmax16(rmax[h], nw);
      // words of slices k-1, k-2, k-3 (from the previous chunk near its start;
      // only read once the first window is complete)
      const uint32_t w1 = j >= 1 ? cur[j - 1][h] : prev[CH - 1][h];
      const uint32_t w2 = j >= 2 ? cur[j - 2][h] : prev[CH + j - 2][h];
      const uint32_t w3 = j >= 3 ? cur[j - 3][h] : prev[CH + j - 3][h];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int p = 2 * h + u;
        const uint32_t x = u ? hi16(nw) : lo16(nw);
        if (FIRST && j < W) {
          st.ws[p] += x;
        } else {
          const uint32_t od = j >= W ? cur[j - W][h] : prev[CH + j - W][h];
          st.ws[p] += x - (u ? hi16(od) : lo16(od));
        }
        if (!FIRST || j >= W - 1) {
          // the window starting at k - 3 wins on a larger sum; on an equal
          // sum the earlier start, already held, has the larger key
          const uint32_t nk = (st.ws[p] << 8) | (uint32_t)(255 - (k0 + j - (W - 1)));
          const bool better = nk > st.key[p];
          st.key[p] = better ? nk : st.key[p];
          st.sv0[p] = better ? (u ? pair16<1>(w3, w2) : pair16<0>(w3, w2)) : st.sv0[p];
          st.sv1[p] = better ? (u ? pair16<1>(w1, nw) : pair16<0>(w1, nw)) : st.sv1[p];
        }
      }
    }
  }
}

template <int PPL, int CH, bool TRACK_MAX>
__device__ __forceinline__ void window_keep(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t sbase, uint32_t stride,
                                            int T, KeepState<PPL>& st, uint32_t (&rmax)[PPL / 2]) {
  constexpr int W = 4;
  static_assert(CH % W == 0 && CH >= W && CH <= 16, "chunk must be a multiple of the window, at most 16");
  constexpr int ND = PPL / 2;
  uint32_t A[CH][ND], B[CH][ND];
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    st.ws[p] = 0; st.key[p] = 0; st.sv0[p] = 0; st.sv1[p] = 0;
  }
  const int nchunk = (T + CH - 1) / CH;
  const int nfull = T / CH;
  load_chunk<PPL, CH>(A, r, voff, sbase, stride, 0);
  if (nchunk > 1) load_chunk<PPL, CH>(B, r, voff, sbase, stride, CH);
  if (nfull >= 1)
    keep_slices<PPL, CH, TRACK_MAX, false, true, 0, CH>(A, A, 0, T, st, rmax);
  else
    keep_slices<PPL, CH, TRACK_MAX, true, true, 0, CH>(A, A, 0, T, st, rmax);
  for (int c = 1; c < nchunk; c += 2) {
    const int k0 = c * CH;
    if (c < nfull) {
      keep_slices<PPL, CH, TRACK_MAX, false, false, 0, W>(B, A, k0, T, st, rmax);
      if (c + 1 < nchunk) load_chunk<PPL, CH>(A, r, voff, sbase, stride, k0 + CH);
      keep_slices<PPL, CH, TRACK_MAX, false, false, W, CH>(B, A, k0, T, st, rmax);
    } else {
      keep_slices<PPL, CH, TRACK_MAX, true, false, 0, CH>(B, A, k0, T, st, rmax);
    }
    if (c + 1 >= nchunk) break;
    const int k1 = k0 + CH;
    if (c + 1 < nfull) {
      keep_slices<PPL, CH, TRACK_MAX, false, false, 0, W>(A, B, k1, T, st, rmax);
      if (c + 2 < nchunk) load_chunk<PPL, CH>(B, r, voff, sbase, stride, k1 + CH);
      keep_slices<PPL, CH, TRACK_MAX, false, false, W, CH>(A, B, k1, T, st, rmax);
    } else {
      keep_slices<PPL, CH, TRACK_MAX, true, false, 0, CH>(A, B, k1, T, st, rmax);
    }
  }
}

// Extraction of one pixel group with its best windows kept: the high gain,
// then, when any lane of the wave owns a switched pixel, the low gain, whose
// window replaces the high-gain one for the switched pixels.  Returns the
// switch mask; st holds the selected gain's windows.
template <int PPL, int CH>
__device__ __forceinline__ uint32_t keep_group(const DevCam& c, __amdgpu_buffer_rsrc_t r, int pix0, int np, int T,
                                               bool dual, KeepState<PPL>& st) {
  uint32_t rmax[PPL / 2];
#pragma unroll
  for (int h = 0; h < PPL / 2; ++h) rmax[h] = 0;
  const uint32_t voff = (uint32_t)pix0 * 2u, stride = (uint32_t)np * 2u;
  uint32_t sw = 0;
  if (dual) {
    window_keep<PPL, CH, true>(r, voff, 0u, stride, T, st, rmax);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const uint32_t m = (p & 1) ? hi16(rmax[p >> 1]) : lo16(rmax[p >> 1]);
      if ((int)m >= c.hg_switch) sw |= 1u << p;
    }
    if (__ballot(sw != 0u)) {
      KeepState<PPL> lg;
      uint32_t unused[PPL / 2];
      window_keep<PPL, CH, false>(r, voff, (uint32_t)T * stride, stride, T, lg, unused);
#pragma unroll
      for (int p = 0; p < PPL; ++p)
        if ((sw >> p) & 1u) {
          st.key[p] = lg.key[p];
          st.sv0[p] = lg.sv0[p];
          st.sv1[p] = lg.sv1[p];
        }
    }
  } else {
    window_keep<PPL, CH, false>(r, voff, 0u, stride, T, st, rmax);
  }
  return sw;
}

// Nt = sum_k k*(256*x[s*+k] - P) and the earliest in-window peak from a kept
// window (samples x0..x3 = low / high halves of sv0, sv1).
__device__ __forceinline__ int32_t kept_nt(uint32_t sv0, uint32_t sv1, int32_t P, int s, int* peak) {
  const uint32_t x[4] = {lo16(sv0), hi16(sv0), lo16(sv1), hi16(sv1)};
  int32_t nt = 0;
  uint32_t pmax = x[0];
  int pk = s;
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    nt += k * (256 * (int32_t)x[k] - P);
    if (x[k] > pmax) { pmax = x[k]; pk = s + k; }
  }
  *peak = pk;
  return nt;
}

// ---------------------------------------------------------------------------
// Window placement by the other extractors.  They produce the same packed key
// (S << 8) | (255 - s*) as the sliding window, so every later step is shared.
// ---------------------------------------------------------------------------
enum : int {
  kExSliding = RTA_EXTRACT_SLIDING,
  kExFixed = RTA_EXTRACT_FIXED,
  kExGlobal = RTA_EXTRACT_GLOBAL_PEAK,
  kExNeighbour = RTA_EXTRACT_NEIGHBOUR_PEAK
};

// Neighbour peak: high-gain slices staged in LDS this many at a time.
constexpr int kNbrRows = 4;

// Sums of the W samples from slice s on of every pixel of the group (one
// load per slice) and, with TRACK_MAX, their packed per-pixel maximum.
template <int PPL, int W, bool TRACK_MAX>
__device__ __forceinline__ void window_at(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t sbase, uint32_t stride,
                                          int s, uint32_t (&S)[PPL], uint32_t (&mx)[PPL / 2]) {
  constexpr int ND = PPL / 2;
  uint32_t d[W][ND];
  uint32_t soff = sbase + (uint32_t)s * stride;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    load_slice<ND>(d[k], r, voff, soff);
    soff += stride;
  }
#pragma unroll
  for (int p = 0; p < PPL; ++p) S[p] = 0;
#pragma unroll
  for (int h = 0; h < ND; ++h) mx[h] = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
#pragma unroll
    for (int h = 0; h < ND; ++h) {
      S[2 * h] += lo16(d[k][h]);
      S[2 * h + 1] += hi16(d[k][h]);
      if constexpr (TRACK_MAX) mx[h] = pkmax16(mx[h], d[k][h]);
    }
  }
}

// Keys of a group whose window start s is known; sw: pixels on low gain.
template <int PPL, int W>
__device__ __forceinline__ void keys_at(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t stride, int T, int s,
                                        const uint32_t (&S_hg)[PPL], uint32_t sw, uint32_t (&key)[PPL]) {
  uint32_t S[PPL];
#pragma unroll
  for (int p = 0; p < PPL; ++p) S[p] = S_hg[p];
  if (__ballot(sw != 0u)) {
    uint32_t SL[PPL], unused[PPL / 2];
    window_at<PPL, W, false>(r, voff, (uint32_t)T * stride, stride, s, SL, unused);
#pragma unroll
    for (int p = 0; p < PPL; ++p)
      if ((sw >> p) & 1u) S[p] = SL[p];
  }
  const uint32_t low = 255u - (uint32_t)s;
#pragma unroll
  for (int p = 0; p < PPL; ++p) key[p] = (S[p] << 8) | low;
}

// Fixed window: samples s0 .. s0+W-1 of every pixel, the gain decided on the
// high-gain samples of that window; nothing else of the trace is read.
template <int PPL, int W>
__device__ __forceinline__ uint32_t fixed_group(const DevCam& c, __amdgpu_buffer_rsrc_t r, int pix0, int np, int T,
                                                bool dual, uint32_t (&key)[PPL]) {
  const uint32_t voff = (uint32_t)pix0 * 2u, stride = (uint32_t)np * 2u;
  const int s0 = c.fixed_start;
  uint32_t S[PPL], mx[PPL / 2];
  window_at<PPL, W, true>(r, voff, 0u, stride, s0, S, mx);
  uint32_t sw = 0;
  if (dual) {
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const uint32_t m = (p & 1) ? hi16(mx[p >> 1]) : lo16(mx[p >> 1]);
      if ((int)m >= c.hg_switch) sw |= 1u << p;
    }
  }
  keys_at<PPL, W>(r, voff, stride, T, s0, S, sw, key);
  return sw;
}

// Sum of v over the wavefront, valid in lane 63, with DPP lane moves only
// (no LDS traffic): pairs and quads by quad permutes, eights and sixteens by
// the half-row and row mirrors, then rows by the row-15 and row-31
// broadcasts (rows outside the row mask add 0).
__device__ __forceinline__ uint32_t wave_sum_u32_last(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

// Global peak, first stage for one group: the wave's sum of the raw
// high-gain samples of pixels below N, slice by slice, added into rows[k]
// (stored on the first pass); returns the group's low-gain bits (full-trace
// raw high-gain maximum >= switch).
template <int PPL, int CH>
__device__ __forceinline__ uint32_t global_rows_group(const DevCam& c, __amdgpu_buffer_rsrc_t r, int pix0, int np,
                                                      int T, bool dual, uint32_t* rows, bool first) {
  constexpr int ND = PPL / 2;
  const uint32_t voff = (uint32_t)pix0 * 2u, stride = (uint32_t)np * 2u;
  const int nv = min(max(c.n_pix - pix0, 0), PPL);
  uint32_t msk[ND], rmax[ND];
#pragma unroll
  for (int h = 0; h < ND; ++h) {
    msk[h] = (2 * h + 1 < nv) ? 0xffffffffu : (2 * h < nv ? 0x0000ffffu : 0u);
    rmax[h] = 0;
  }
  const bool writer = (threadIdx.x & (kWave - 1)) == kWave - 1;
  uint32_t A[CH][ND];
  for (int k0 = 0; k0 < T; k0 += CH) {
    load_chunk<PPL, CH>(A, r, voff, 0u, stride, k0);
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (k0 + j >= T) continue;
      uint32_t v = 0;
#pragma unroll
      for (int h = 0; h < ND; ++h) {
        const uint32_t x = A[j][h] & msk[h];
        v += lo16(x) + hi16(x);
        rmax[h] = pkmax16(rmax[h], x);
      }
      v = wave_sum_u32_last(v);
      if (writer) rows[k0 + j] = first ? v : rows[k0 + j] + v;
    }
  }
  uint32_t sw = 0;
  if (dual) {
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const uint32_t m = (p & 1) ? hi16(rmax[p >> 1]) : lo16(rmax[p >> 1]);
      if ((int)m >= c.hg_switch) sw |= 1u << p;
    }
  }
  return sw;
}

// Global peak start: the earliest maximiser of C(s) = sum_{k<W} of the
// camera-summed slices, from the per-wave partial sums rows[w * 256 + k].
// Called by every thread of the block (contains a barrier).
template <int NT, int W>
__device__ __forceinline__ int global_start(const uint32_t* rows, int T, int32_t* start) {
  constexpr int NW = NT / kWave;
  if (threadIdx.x < kWave) {
    uint64_t best = 0;
    for (int s = threadIdx.x; s + W <= T; s += kWave) {
      uint64_t C = 0;
#pragma unroll
      for (int k = 0; k < W; ++k)
#pragma unroll
        for (int w = 0; w < NW; ++w) C += rows[w * 256 + s + k];
      const uint64_t cand = (C << 8) | (uint64_t)(255 - s);
      best = cand > best ? cand : best;
    }
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) {
      const uint64_t o = __shfl_xor(best, off, kWave);
      best = o > best ? o : best;
    }
    if (threadIdx.x == 0) *start = 255 - (int)(best & 255u);
  }
  __syncthreads();
  return *start;
}

// Neighbour peak for every pixel of the event: the earliest maximiser of
// C_i(s) = sum over the neighbours j of i of the raw high-gain window sum
// W_j(s).  Four high-gain slices at a time are staged in LDS transposed,
// one 64-bit word of four halfwords per pixel (slices k0..k0+3; word Npad = 0
// stands in for a missing neighbour), so a pixel's neighbours cost one 8-byte
// read each per four slices, and the per-slice neighbour sums y(t) come from
// packed dot products.  The next four slices are loaded while the current
// ones are used.  Words sit at the pixels' lattice-row positions, and in this
// stage lane t takes positions t, t + NT, ...: the lanes of one read are
// neighbours along a row, so each direction's neighbour words are (nearly)
// consecutive; the pixels' best keys then go through LDS to the lanes'
// PPL-pixel groups.  Each lane keeps, for each of its pixels, the last
// W-1 sums to form C(t-W+1), the best key (C << 8) | (255 - s) and the raw
// high-gain maximum (gain decision on the whole trace, as for the sliding
// window); a step whose four slices all end a window inside the trace forms
// its four window sums at once.  Then the pixel's own W samples at its start
// on its selected gain give S.  Called by every thread of the block
// (contains barriers).
template <int PPL, int W, int NT, class Fn>
__device__ __forceinline__ void neighbour_event(const DevCam& c, __amdgpu_buffer_rsrc_t r,
                                                const uint16_t* __restrict__ ev, uint16_t* xrow, uint32_t* keys,
                                                Fn&& fn) {
  static_assert(kNbrRows == 4, "four slices per staged pixel word pair");
  constexpr int MAXK = (kMaxPix + NT - 1) / NT;  // pixels per lane: t, t + NT, ...
  constexpr int MAXP = (kMaxPix + NT * PPL - 1) / (NT * PPL);
  const int N = c.n_pix, np = c.n_pix_pad, T = c.n_samp;
  const bool dual = c.n_gain == 2;
  const int npass = (N + NT * PPL - 1) / (NT * PPL);
  // staged words: slices k0, k0+1 in the low dword, k0+2, k0+3 in the high
  // one (64-bit words: the packed dot of a two-lane vector's second element
  // has been seen compiled onto its first)
  uint64_t* xs = reinterpret_cast<uint64_t*>(xrow);
  // position p = 8 g + m lives in word 8 g + (m ^ (g & 7)): consecutive
  // lanes reading consecutive positions touch distinct banks
  auto slot = [](uint32_t j) { return (j & ~7u) | ((j ^ (j >> 3)) & 7u); };
  uint32_t nb[MAXK][3];  // six neighbour words per position: LDS byte offsets, 16 bits each (word Npad if missing)
  uint32_t ring[MAXK][W - 1];
  uint32_t best[MAXK], hmax2[MAXK];
#pragma unroll
  for (int k = 0; k < MAXK; ++k) {
    const int p = (int)threadIdx.x + k * NT;
    nb[k][0] = nb[k][1] = nb[k][2] = (uint32_t)np * 8u * 0x10001u;
    if (p < N) {
      const int4 v = *reinterpret_cast<const int4*>(c.lat + (size_t)p * kNbrCols);
      const uint32_t w3[3] = {(uint32_t)v.x, (uint32_t)v.y, (uint32_t)v.z};
#pragma unroll
      for (int h = 0; h < 3; ++h) {
        const uint32_t lo = (w3[h] & 0x8000u) ? (uint32_t)np : slot(w3[h] & 0xffffu);
        const uint32_t hi = (w3[h] & 0x80000000u) ? (uint32_t)np : slot(w3[h] >> 16);
        nb[k][h] = (lo << 3) | (hi << 19);  // (Npad + 1) * 8 bytes < 2^16
      }
    }
#pragma unroll
    for (int u = 0; u < W - 1; ++u) ring[k][u] = 0;
    best[k] = 0;
    hmax2[k] = 0;
  }
  if (threadIdx.x == 0) xs[np] = 0ull;
  // thread q stages 16-byte pixel group q (np / 8 <= kMaxPix / 8 <= NT
  // groups), the next four slices loaded while the current ones are used
  static_assert(kMaxPix / 8 <= NT, "one staged pixel group per thread");
  const int q = threadIdx.x;
  const bool stager = q < np / 8;
  const us2 row_lo = {1, 0}, row_hi = {0, 1};
  // the words of this thread's eight pixels, at their positions
  uint32_t dst[8];
  if (stager) {
    const int4 lp = *reinterpret_cast<const int4*>(c.lpos + (size_t)q * 8);
    const uint32_t w4[4] = {(uint32_t)lp.x, (uint32_t)lp.y, (uint32_t)lp.z, (uint32_t)lp.w};
#pragma unroll
    for (int m = 0; m < 8; ++m) dst[m] = slot((w4[m >> 1] >> ((m & 1) * 16)) & 0xffffu);
  }
  u32x4 d[kNbrRows];
  auto load4 = [&](int k0) {
#pragma unroll
    for (int k = 0; k < kNbrRows; ++k)
      d[k] = __builtin_amdgcn_raw_buffer_load_b128(r, q * 16, (k0 + k) * np * 2, RTA_TRACE_CPOL);
  };
  if (stager) load4(0);
  for (int k0 = 0; k0 < T; k0 += kNbrRows) {
    // keep the neighbour offsets packed: unpacked out of the loop they
    // would take six registers per position instead of three
#pragma unroll
    for (int k = 0; k < MAXK; ++k)
#pragma unroll
      for (int h = 0; h < 3; ++h) asm volatile("" : "+v"(nb[k][h]));
    __syncthreads();  // the previous slices are consumed
    if (stager) {
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const uint32_t sel = (m & 1) ? 0x07060302u : 0x05040100u;  // high / low halfwords
        xs[dst[m]] = (uint64_t)__builtin_amdgcn_perm(d[1][m >> 1], d[0][m >> 1], sel) |
                                    ((uint64_t)__builtin_amdgcn_perm(d[3][m >> 1], d[2][m >> 1], sel) << 32);
      }
    }
    __syncthreads();
    if (stager && k0 + kNbrRows < T) load4(k0 + kNbrRows);
    // uniform: every slice of this step has a full window inside the trace
    const bool full = k0 >= W - 1 && k0 + kNbrRows <= T;
    const uint32_t key0 = (uint32_t)(255 - (k0 - (W - 1)));  // 255 - window start of slice k0
#pragma unroll
    for (int k = 0; k < MAXK; ++k) {
      const int p = (int)threadIdx.x + k * NT;
      if (p >= N) continue;
      uint64_t v[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        const uint32_t off = (nb[k][m >> 1] >> ((m & 1) * 16)) & 0xffffu;
        v[m] = *reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(xs) + off);
      }
      // the six neighbours' slices summed two at a time in saturating 16-bit
      // halves; a sum that reached 65535 (so maybe more) is formed again in
      // 32 bits, for the whole wave when any lane needs it
      us2 s01 = __builtin_bit_cast(us2, (uint32_t)v[0]), s23 = __builtin_bit_cast(us2, (uint32_t)(v[0] >> 32));
#pragma unroll
      for (int m = 1; m < 6; ++m) {
        s01 = __builtin_elementwise_add_sat(s01, __builtin_bit_cast(us2, (uint32_t)v[m]));
        s23 = __builtin_elementwise_add_sat(s23, __builtin_bit_cast(us2, (uint32_t)(v[m] >> 32)));
      }
      const us2 smax = __builtin_elementwise_max(s01, s23);
      uint32_t y[kNbrRows] = {s01[0], s01[1], s23[0], s23[1]};
      if (__ballot(smax[0] == 0xffffu || smax[1] == 0xffffu)) {
#pragma unroll
        for (int u = 0; u < kNbrRows; ++u) y[u] = 0;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          const uint32_t v01 = (uint32_t)v[m], v23 = (uint32_t)(v[m] >> 32);
          y[0] = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v01), row_lo, y[0], false);
          y[1] = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v01), row_hi, y[1], false);
          y[2] = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v23), row_lo, y[2], false);
          y[3] = __builtin_amdgcn_udot2(__builtin_bit_cast(us2, v23), row_hi, y[3], false);
        }
      }
      const uint64_t own = xs[slot((uint32_t)p)];
      const uint32_t o01 = (uint32_t)own, o23 = (uint32_t)(own >> 32);
      if constexpr (W == kNbrRows) if (full) {
        // all four slices inside the trace and past the first window: the
        // four window sums C(k0 + u) = y(k0 + u - 3) + ... + y(k0 + u) from
        // the ring (ring[z] = y(k0 - 1 - z)) and this step's sums, the
        // ring shifted once, the high-gain maximum on packed halfwords
        const us2 hm = __builtin_elementwise_max(
            __builtin_elementwise_max(__builtin_bit_cast(us2, hmax2[k]), __builtin_bit_cast(us2, o01)),
            __builtin_bit_cast(us2, o23));
        hmax2[k] = __builtin_bit_cast(uint32_t, hm);
        const uint32_t r01 = ring[k][0] + ring[k][1], y01 = y[0] + y[1];
        const uint32_t C0 = y[0] + r01 + ring[k][2], C1 = y[1] + y[0] + r01;
        const uint32_t C2 = y[2] + y01 + ring[k][0], C3 = y[3] + y[2] + y01;
        best[k] = max(best[k], (C0 << 8) | key0);
        best[k] = max(best[k], (C1 << 8) | (key0 - 1u));
        best[k] = max(best[k], (C2 << 8) | (key0 - 2u));
        best[k] = max(best[k], (C3 << 8) | (key0 - 3u));
        ring[k][0] = y[3];
        ring[k][1] = y[2];
        ring[k][2] = y[1];
        continue;
      }
      const uint32_t xo[kNbrRows] = {lo16(o01), hi16(o01), lo16(o23), hi16(o23)};
#pragma unroll
      for (int u = 0; u < kNbrRows; ++u) {
        const int t = k0 + u;
        if (t >= T) break;
        hmax2[k] = max(hmax2[k] & 0xffffu, xo[u]) | (hmax2[k] & 0xffff0000u);
        uint32_t C = y[u];
#pragma unroll
        for (int z = 0; z < W - 1; ++z) C += ring[k][z];
        if (t >= W - 1) best[k] = max(best[k], (C << 8) | (uint32_t)(255 - (t - (W - 1))));
#pragma unroll
        for (int z = W - 2; z > 0; --z) ring[k][z] = ring[k][z - 1];
        ring[k][0] = y[u];
      }
    }
  }
  // hand the keys over to the lanes' pixel groups: the best key of each
  // pixel (C < 2^21, so bits 29..31 are free) with bit 31 = low gain
#pragma unroll
  for (int k = 0; k < MAXK; ++k) {
    const int p = (int)threadIdx.x + k * NT;
    const uint32_t hm = max(lo16(hmax2[k]), hi16(hmax2[k]));
    if (p < N) {
      const uint32_t pix = (uint32_t)c.lat[(size_t)p * kNbrCols + 6] & 0xffffu;  // the pixel at position p
      keys[pix] = best[k] | ((dual && (int)hm >= c.hg_switch) ? 0x80000000u : 0u);
    }
  }
  __syncthreads();
#pragma unroll
  for (int ps = 0; ps < MAXP; ++ps) {
    if (ps >= npass) continue;
    const int pix0 = (ps * NT + (int)threadIdx.x) * PPL;
    uint32_t sw = 0, key[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const int i = pix0 + p;
      key[p] = 0;
      if (i >= N) continue;
      const uint32_t kb = keys[i];
      const int g = (int)(kb >> 31);
      sw |= (uint32_t)g << p;
      const int s = 255 - (int)(kb & 255u);
      const uint16_t* col = ev + ((size_t)g * T + s) * np + i;
      uint32_t S = 0;
#pragma unroll
      for (int u = 0; u < W; ++u) S += col[(size_t)u * np];
      key[p] = (S << 8) | (uint32_t)(255 - s);
    }
    fn(pix0, key, sw);
  }
}

// Keys of every pixel of one event, group by group: fn(pix0, key, sw) for
// each of this thread's groups.  rows / start: LDS scratch of the global
// peak (NT/64 * 256 words, one word); xrow: LDS slices of the neighbour
// peak (kNbrRows * (kMaxPix + 8) halfwords).
template <int EX, int PPL, int W, int CH, int NT, class Fn>
__device__ __forceinline__ void extract_event(const DevCam& c, __amdgpu_buffer_rsrc_t r, const uint16_t* ev,
                                              uint32_t* rows, int32_t* start, uint16_t* xrow, Fn&& fn) {
  const int N = c.n_pix, np = c.n_pix_pad, T = c.n_samp;
  const bool dual = c.n_gain == 2;
  // Uniform pass loop: every lane streams (loads past the event read 0 from
  // the bounds-checked buffer); the callback guards its stores.
  const int npass = (N + NT * PPL - 1) / (NT * PPL);
  if constexpr (EX == kExSliding || EX == kExFixed) {
    for (int ps = 0; ps < npass; ++ps) {
      const int pix0 = (ps * NT + (int)threadIdx.x) * PPL;
      uint32_t key[PPL];
      uint32_t sw;
      if constexpr (EX == kExSliding)
        sw = extract_group<PPL, W, CH>(c, r, pix0, np, T, dual, key);
      else
        sw = fixed_group<PPL, W>(c, r, pix0, np, T, dual, key);
      fn(pix0, key, sw);
    }
  } else if constexpr (EX == kExNeighbour) {
    neighbour_event<PPL, W, NT>(c, r, ev, xrow, rows, fn);
  } else {
    constexpr int MAXP = (kMaxPix + NT * PPL - 1) / (NT * PPL);
    uint32_t* my_rows = rows + (threadIdx.x / kWave) * 256;
    uint32_t swp[MAXP];
#pragma unroll
    for (int ps = 0; ps < MAXP; ++ps) {
      swp[ps] = 0;
      if (ps < npass)
        swp[ps] = global_rows_group<PPL, CH>(c, r, (ps * NT + (int)threadIdx.x) * PPL, np, T, dual, my_rows,
                                             ps == 0);
    }
    __syncthreads();
    const int s = global_start<NT, W>(rows, T, start);
    const uint32_t stride = (uint32_t)np * 2u;
#pragma unroll
    for (int ps = 0; ps < MAXP; ++ps) {
      if (ps < npass) {
        const int pix0 = (ps * NT + (int)threadIdx.x) * PPL;
        const uint32_t voff = (uint32_t)pix0 * 2u;
        uint32_t S[PPL], unused[PPL / 2], key[PPL];
        window_at<PPL, W, false>(r, voff, 0u, stride, s, S, unused);
        keys_at<PPL, W>(r, voff, stride, T, s, S, swp[ps], key);
        fn(pix0, key, swp[ps]);
      }
    }
  }
}

// D = 256*S - w*P from the packed key.
template <int W>
__device__ __forceinline__ int32_t key_to_d(uint32_t key, int32_t P) {
  return (int32_t)(key & 0xFFFFFF00u) - W * P;
}

// Time numerator Nt = sum_k k*(256*x[s+k] - P) and the in-window peak index
// from the window samples (re-read from the trace).
template <int W>
__device__ __forceinline__ int32_t window_nt(const uint16_t* __restrict__ col, int np, int s, int32_t P, int* peak) {
  int32_t nt = 0;
  uint32_t pmax = col[(size_t)s * np];
  int pk = s;
#pragma unroll
  for (int k = 1; k < W; ++k) {
    const uint32_t x = col[(size_t)(s + k) * np];
    nt += k * (256 * (int32_t)x - P);
    if (x > pmax) { pmax = x; pk = s + k; }
  }
  if (peak) *peak = pk;
  return nt;
}

// Peak time t = s* + Nt/D (window centre when D <= 0), evaluated in FP64.
template <int W>
__device__ __forceinline__ double peak_time(int s, int32_t nt, int32_t d) {
  return d > 0 ? (double)s + (double)nt / (double)d : (double)s + 0.5 * (double)(W - 1);
}

__device__ __forceinline__ uint32_t pixel_flag(const DevCam& c, int g, int i, int32_t d) {
  const int o = g * c.n_pix_pad + i;
  return (uint32_t)(d >= c.thr_bnd[o]) | ((uint32_t)(d >= c.thr_pic[o]) << 1);
}

// The same with given levels (p.e.): the thresholds ceil(256 a T) formed in
// FP64 in the order the camera creation forms its tables (256 a is exact,
// then one rounded product), so the levels the camera was made with give
// its tables' values.  The host bounds them to |.| <= 2e9.
__device__ __forceinline__ uint32_t pixel_flag_at(const DevCam& c, int g, int i, int32_t d, float t_pic,
                                                  float t_bnd) {
  const double a256 = 256.0 * (double)c.a[g * c.n_pix_pad + i];
  const int32_t tp = (int32_t)ceil(a256 * (double)t_pic), tb = (int32_t)ceil(a256 * (double)t_bnd);
  return (uint32_t)(d >= tb) | ((uint32_t)(d >= tp) << 1);
}

// ---------------------------------------------------------------------------
// Workgroup-shared state of one camera event.
// ---------------------------------------------------------------------------
struct TelSmem {
  union {
    uint32_t key[kMaxPix];   // (S << 8) | (255 - s*) per pixel; reused as union-find parents
    uint32_t rows[kMaxPix];  // global peak: per-wave slice sums; neighbour peak: key hand-over (extraction only)
  };
  uint8_t flag[kMaxPix];     // bit 0: D >= Tb, bit 1: D >= Tp, bit 2: low gain
  uint64_t mbits[kMaxWords]; // cleaning mask, one word per 64 pixels
  int32_t wbase[kMaxWords + 1];
  uint16_t list[kMaxPix];    // slot -> pixel | gain << 15
  union alignas(16) {        // 16-byte aligned: slices are staged with 16-byte stores
    struct {
      // per slot, fused path: D and Nt in their low 28 bits (both fit in 28
      // signed bits), s* split over the top 4 bits of each; unfused path:
      // D in dq, the float bits of the given peak time in nt
      uint32_t dq[kMaxPix];
      uint32_t nt[kMaxPix];
    } slot;
    uint16_t xrow[kNbrRows * (kMaxPix + 8)];  // neighbour peak: staged slices + zero slot (extraction only)
  };
  double red[16 * 8];        // cross-wave reduction scratch
  int32_t nlow_w[16];        // per-wave counts of low-gain pixels
  int32_t start;             // global peak window start
};

__device__ __forceinline__ int32_t sext28(uint32_t v) { return (int32_t)(v << 4) >> 4; }

// Charge of slot j: q = D / (256 a), formed where it is used (the same float
// every time, and the float the calibration writes as q); on the unfused
// path the given q.
template <bool FUSED>
__device__ __forceinline__ float slot_q(const DevCam& c, const TelSmem& sm, int j, int i) {
  if constexpr (FUSED) {
    const int g = sm.list[j] >> 15;
    return (float)sext28(sm.slot.dq[j]) / (256.0f * c.a[g * c.n_pix_pad + i]);
  } else {
    return __uint_as_float(sm.slot.dq[j]);
  }
}

// Peak time of slot j (samples): s* + Nt / D from the packed slot, or the
// given float time on the unfused path.
template <bool FUSED, int W>
__device__ __forceinline__ double slot_t(const TelSmem& sm, int j) {
  const uint32_t a = sm.slot.dq[j], b = sm.slot.nt[j];
  if constexpr (FUSED) {
    const int s = (int)(((a >> 28) << 4) | (b >> 28));
    return peak_time<W>(s, sext28(b), sext28(a));
  } else {
    return (double)__uint_as_float(b);
  }
}

template <typename T, int NV, int NT>
__device__ __forceinline__ void block_sum(T (&v)[NV], double* red_raw) {
  T* red = reinterpret_cast<T*>(red_raw);
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, kWave);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    T s = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w * NV + k];
    v[k] = s;
  }
  __syncthreads();
}

// The same sums over one wavefront (the other wavefronts hold nothing): the
// butterfly of block_sum, then its cross-wave sum, here 0 + the wave's sum.
template <typename T, int NV>
__device__ __forceinline__ void wave_sum(T (&v)[NV]) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, kWave);
    v[k] = T(0) + v[k];
  }
}

// Workgroup total of a per-thread count: each wavefront's sum goes to
// sm.nlow_w before a barrier the caller provides; total_count reads them
// after it.
__device__ __forceinline__ void post_count(TelSmem& sm, int v) {
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) sm.nlow_w[threadIdx.x / kWave] = v;
}

template <int NT>
__device__ __forceinline__ int total_count(const TelSmem& sm) {
  int s = 0;
#pragma unroll
  for (int w = 0; w < NT / kWave; ++w) s += sm.nlow_w[w];
  return s;
}

__device__ __forceinline__ bool mask_bit(const TelSmem& sm, int i) { return (sm.mbits[i >> 6] >> (i & 63)) & 1ull; }

__device__ __forceinline__ int mask_slot(const TelSmem& sm, int i) {
  const uint64_t w = sm.mbits[i >> 6];
  return sm.wbase[i >> 6] + __popcll(w & ((1ull << (i & 63)) - 1ull));
}

// Phase 1 (fused): extraction of all pixels into LDS.  Returns this thread's
// count of low-gain pixels.
template <int EX, int PPL, int W, int CH, int NT>
__device__ __forceinline__ int extract_phase(const DevCam& c, const uint16_t* __restrict__ ev, TelSmem& sm) {
  const int N = c.n_pix, np = c.n_pix_pad;
  const __amdgpu_buffer_rsrc_t r = event_rsrc(ev, c.event_elems);
  int nlow = 0;
  extract_event<EX, PPL, W, CH, NT>(c, r, ev, sm.rows, &sm.start, sm.xrow, [&](int pix0, const uint32_t (&key)[PPL],
                                                                                uint32_t sw) {
    if (pix0 >= N) return;
    int32_t P[PPL], Tb[PPL], Tp[PPL];
    load_i32<PPL>(P, c.P256 + pix0);
    load_i32<PPL>(Tb, c.thr_bnd + pix0);
    load_i32<PPL>(Tp, c.thr_pic + pix0);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const int i = pix0 + p;
      if (i < N) {
        const int g = (sw >> p) & 1u;
        int32_t Pv = P[p], tb = Tb[p], tp = Tp[p];
        if (g) { Pv = c.P256[np + i]; tb = c.thr_bnd[np + i]; tp = c.thr_pic[np + i]; }
        const int32_t d = key_to_d<W>(key[p], Pv);
        sm.key[i] = key[p];
        sm.flag[i] = (uint8_t)((uint32_t)(d >= tb) | ((uint32_t)(d >= tp) << 1) | ((uint32_t)g << 2));
        nlow += g;
      }
    }
  });
  return nlow;
}

// Phase 2: mask words from the flags (needs flags of all pixels).
template <int NT>
__device__ __forceinline__ void mask_phase(const DevCam& c, TelSmem& sm) {
  const int N = c.n_pix, nw = (N + 63) >> 6;
  const int lane = threadIdx.x & (kWave - 1);
  for (int base = threadIdx.x & ~(kWave - 1); base < nw * kWave; base += NT) {
    const int i = base + lane;
    bool m = false;
    if (i < N) {
      const uint32_t f = sm.flag[i] & 3u;
      if (f) {
        const int4 nv = *reinterpret_cast<const int4*>(c.nbr + (size_t)i * kNbrCols);
        const int16_t* nb = reinterpret_cast<const int16_t*>(&nv);
        uint32_t any = 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const int j = nb[k];
          if (j >= 0) any |= sm.flag[j];
        }
        m = ((f & 1u) && (any & 2u)) || ((f & 2u) && (any & 1u));
      }
    }
    const uint64_t b = __ballot(m);
    if (lane == 0) sm.mbits[base >> 6] = b;
  }
}

// Phase 3: exclusive prefix of the mask-word popcounts (one wavefront).
__device__ __forceinline__ void scan_phase(int N, TelSmem& sm) {
  const int nw = (N + 63) >> 6;
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    const int cnt = lane < nw ? __popcll(sm.mbits[lane]) : 0;
    int inc = cnt;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int o = __shfl_up(inc, off, kWave);
      if (lane >= off) inc += o;
    }
    if (lane < nw) sm.wbase[lane] = inc - cnt;
    if (lane == nw - 1) sm.wbase[nw] = inc;
  }
}

// Phase 4: slot list of cleaned pixels with q, x, y, t.  FUSED takes D /
// gain / s* from LDS and re-reads the window samples for t; otherwise D,
// gain and t come from global arrays of this event.
template <int NT, int W, bool FUSED>
__device__ __forceinline__ void list_phase(const DevCam& c, TelSmem& sm, const uint16_t* __restrict__ ev,
                                           const float* __restrict__ qg, const int32_t* __restrict__ Dg,
                                           const uint8_t* __restrict__ gg, const float* __restrict__ tg) {
  const int N = c.n_pix, nw = (N + 63) >> 6, np = c.n_pix_pad;
  const int lane = threadIdx.x & (kWave - 1);
  for (int base = threadIdx.x & ~(kWave - 1); base < nw * kWave; base += NT) {
    const int i = base + lane;
    const uint64_t bits = sm.mbits[base >> 6];
    if ((bits >> lane) & 1ull) {
      const int j = sm.wbase[base >> 6] + __popcll(bits & ((1ull << lane) - 1ull));
      if constexpr (FUSED) {
        const uint32_t k = sm.key[i];
        const int g = (int)(sm.flag[i] >> 2);
        const int s = 255 - (int)(k & 255u);
        const int32_t P = c.P256[g * np + i];
        const int32_t d = key_to_d<W>(k, P);
        const int32_t nt = window_nt<W>(ev + (size_t)g * c.n_samp * np + i, np, s, P, nullptr);
        sm.list[j] = (uint16_t)(i | (g << 15));
        sm.slot.dq[j] = ((uint32_t)d & 0x0FFFFFFFu) | ((uint32_t)(s >> 4) << 28);
        sm.slot.nt[j] = ((uint32_t)nt & 0x0FFFFFFFu) | ((uint32_t)(s & 15) << 28);
      } else {
        // the given charge, or D / (256 a) formed as the calibration forms q
        const int g = gg ? (int)gg[i] : 0;
        const float q = qg ? qg[i] : (float)Dg[i] / (256.0f * c.a[g * np + i]);
        sm.list[j] = (uint16_t)(i | (g << 15));
        sm.slot.dq[j] = __float_as_uint(q);
        sm.slot.nt[j] = __float_as_uint(tg[i]);
      }
    }
  }
}

__device__ __forceinline__ int uf_find(volatile int32_t* par, int x) {
  int p = par[x];
  while (p != x) {
    x = p;
    p = par[x];
  }
  return x;
}

// Hooks the larger root under the smaller; a root changes only by a CAS from
// itself to a smaller index, so parents strictly decrease and find ends.
__device__ __forceinline__ void uf_union(int32_t* par, int a, int b) {
  volatile int32_t* vp = par;
  for (;;) {
    a = uf_find(vp, a);
    b = uf_find(vp, b);
    if (a == b) return;
    if (a < b) { const int t = a; a = b; b = t; }
    if (atomicCAS(&par[a], a, b) == a) return;
  }
}

// Phase 5: islands = roots of the union-find forest over mask slots.
// Returns this thread's root count.  The per-pixel keys (no longer needed)
// hold the parents.  WAVE: wavefront 0 alone, over at most 64 slots, the
// barriers replaced by wavefront-scope ordering of its LDS accesses.
template <int NT, bool WAVE>
__device__ __forceinline__ int islands_phase(const DevCam& c, TelSmem& sm, int n) {
  constexpr int STEP = WAVE ? kWave : NT;
  int32_t* par = reinterpret_cast<int32_t*>(sm.key);
  for (int j = threadIdx.x; j < n; j += STEP) par[j] = j;
  if constexpr (WAVE)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  else
    __syncthreads();
  for (int j = threadIdx.x; j < n; j += STEP) {
    const int i = sm.list[j] & 0x7FFF;
    const int4 nv = *reinterpret_cast<const int4*>(c.nbr + (size_t)i * kNbrCols);
    const int16_t* nb = reinterpret_cast<const int16_t*>(&nv);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int m = nb[k];
      if (m > i && mask_bit(sm, m)) uf_union(par, j, mask_slot(sm, m));
    }
  }
  if constexpr (WAVE)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  else
    __syncthreads();
  int roots = 0;
  for (int j = threadIdx.x; j < n; j += STEP) roots += (((volatile int32_t*)par)[j] == j);
  return roots;
}

// Phase 6: Hillas reductions and the record.
// Centre of gravity and second moments are FP32 sums of centred terms.  The
// third pass takes the longitudinal and transverse coordinates l, w in the
// rotated frame: skewness and kurtosis from q l^3, q l^4, the width from the
// minor-axis moment q w^2 (exact for collinear pixels, unlike
// sqrt(det / l+), which keeps only half the digits when the width is small),
// and the time regression from the FP64 sums of l, l^2, t and l t (times are
// absolute sample numbers, so FP32 would cancel most digits of small time
// gradients; in FP64 the centring cancels about t / spread(t) x mean(l) /
// spread(l) digits, harmless).
template <int NT, int W, bool FUSED, bool WAVE>
__device__ __forceinline__ rta_hillas_rec hillas_phase(const DevCam& c, TelSmem& sm, int n, int roots, int nlow) {
  constexpr int STEP = WAVE ? kWave : NT;
  float v1[5] = {0.f, 0.f, 0.f, 0.f, (float)roots};
  for (int j = threadIdx.x; j < n; j += STEP) {
    const int i = sm.list[j] & 0x7FFF;
    const float q = slot_q<FUSED>(c, sm, j, i);
    v1[0] += q;
    v1[1] += q * c.x[i];
    v1[2] += q * c.y[i];
    if (c.border[i]) v1[3] += q;
  }
  if constexpr (WAVE)
    wave_sum(v1);
  else
    block_sum<float, 5, NT>(v1, sm.red);
  const float S = v1[0];
  rta_hillas_rec r;
  r.size = S;
  r.n_pix = n;
  r.n_islands = (int32_t)v1[4];
  r.n_lowgain = nlow;
  r.flags = r.n_lowgain > 0 ? RTA_FLAG_LOW_GAIN : 0u;
  if (n < 2 || !(S > 0.f)) {
    r.cog_x = r.cog_y = r.length = r.width = r.psi = r.skewness = r.kurtosis = kNaN;
    r.time_gradient = r.time_intercept = r.leakage = r.cog_dist = kNaN;
    r.flags |= RTA_FLAG_HILLAS_INVALID | RTA_FLAG_TIME_INVALID;
    return r;
  }
  const float xm = v1[1] / S, ym = v1[2] / S;
  float v2[3] = {0.f, 0.f, 0.f};
  for (int j = threadIdx.x; j < n; j += STEP) {
    const int i = sm.list[j] & 0x7FFF;
    const float q = slot_q<FUSED>(c, sm, j, i), dx = c.x[i] - xm, dy = c.y[i] - ym;
    v2[0] += q * dx * dx;
    v2[1] += q * dy * dy;
    v2[2] += q * dx * dy;
  }
  if constexpr (WAVE)
    wave_sum(v2);
  else
    block_sum<float, 3, NT>(v2, sm.red);
  const float sxx = v2[0] / S, syy = v2[1] / S, sxy = v2[2] / S;
  const float hd = 0.5f * (sxx - syy);
  const float lp = 0.5f * (sxx + syy) + sqrtf(hd * hd + sxy * sxy);
  float psi = 0.5f * atan2f(2.0f * sxy, sxx - syy);
  if (psi <= -0.5f * (float)M_PI) psi += (float)M_PI;
  const float len = sqrtf(lp);
  const float cs = cosf(psi), sn = sinf(psi);
  // l of slot 0: every l equal to it (fewer than two distinct l) leaves the
  // time gradient undefined
  float l0;
  {
    const int i = sm.list[0] & 0x7FFF;
    l0 = (c.x[i] - xm) * cs + (c.y[i] - ym) * sn;
  }
  // q l^3, q l^4, q w^2, l, l^2, t, l t, |l - l0|
  double v3[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < n; j += STEP) {
    const int i = sm.list[j] & 0x7FFF;
    const float q = slot_q<FUSED>(c, sm, j, i), dx = c.x[i] - xm, dy = c.y[i] - ym;
    const float l = dx * cs + dy * sn;
    const float w = dy * cs - dx * sn;
    const float l2 = l * l;
    v3[0] += (double)(q * l2 * l);
    v3[1] += (double)(q * l2 * l2);
    v3[2] += (double)(q * w * w);
    const double ld = (double)l, td = slot_t<FUSED, W>(sm, j);
    v3[3] += ld;
    v3[4] += ld * ld;
    v3[5] += td;
    v3[6] += ld * td;
    v3[7] += fabs(ld - (double)l0);
  }
  if constexpr (WAVE)
    wave_sum(v3);
  else
    block_sum<double, 8, NT>(v3, sm.red);
  const double nd = (double)n, lbar = v3[3] / nd, tbar = v3[5] / nd;
  const double sll = v3[4] - v3[3] * lbar, slt = v3[6] - v3[3] * tbar;
  r.cog_x = xm;
  r.cog_y = ym;
  r.length = len;
  r.width = sqrtf(fmaxf((float)v3[2] / S, 0.f));
  r.psi = psi;
  const float len3 = len * len * len;
  r.skewness = (float)v3[0] / (S * len3);
  r.kurtosis = (float)v3[1] / (S * len3 * len);
  r.leakage = v1[3] / S;
  r.cog_dist = sqrtf(xm * xm + ym * ym);
  if (v3[7] > 0.0 && sll > 0.0) {
    const double g = slt / sll;
    r.time_gradient = (float)g;
    r.time_intercept = (float)(tbar - g * lbar);
  } else {
    r.time_gradient = r.time_intercept = kNaN;
    r.flags |= RTA_FLAG_TIME_INVALID;
  }
  return r;
}

// Phases 5 and 6 over the n mask slots; nlow: the image's low-gain pixel
// count.  An image of at most 64 mask pixels (most images) is done by
// wavefront 0 alone, with no barrier, while the other wavefronts return an
// unused record at once; the sums are the same bit for bit, since the other
// wavefronts would contribute exact zeros.  The threads of wavefront 0
// return the record.
template <int NT, int W, bool FUSED>
__device__ __forceinline__ rta_hillas_rec islands_hillas(const DevCam& c, TelSmem& sm, int n, int nlow) {
  if (n <= kWave) {
    if (threadIdx.x >= kWave) return rta_hillas_rec{};
    const int roots = islands_phase<NT, true>(c, sm, n);
    return hillas_phase<NT, W, FUSED, true>(c, sm, n, roots, nlow);
  }
  const int roots = islands_phase<NT, false>(c, sm, n);
  return hillas_phase<NT, W, FUSED, false>(c, sm, n, roots, nlow);
}

// Calibration -> cleaning -> Hillas of one camera event; the threads of
// wavefront 0 return the record.
template <int EX, int PPL, int W, int CH, int NT>
__device__ __forceinline__ rta_hillas_rec process_telescope(const DevCam& c, const uint16_t* __restrict__ ev,
                                                            TelSmem& sm) {
  post_count(sm, extract_phase<EX, PPL, W, CH, NT>(c, ev, sm));
  __syncthreads();
  mask_phase<NT>(c, sm);
  __syncthreads();
  scan_phase(c.n_pix, sm);
  __syncthreads();
  const int n = sm.wbase[(c.n_pix + 63) >> 6];
  list_phase<NT, W, true>(c, sm, ev, nullptr, nullptr, nullptr, nullptr);
  __syncthreads();
  return islands_hillas<NT, W, true>(c, sm, n, total_count<NT>(sm));
}

__device__ __forceinline__ void bad_record(rta_hillas_rec* out) {
  rta_hillas_rec r;
  r.size = r.cog_x = r.cog_y = r.length = r.width = r.psi = r.skewness = r.kurtosis = kNaN;
  r.time_gradient = r.time_intercept = r.leakage = r.cog_dist = kNaN;
  r.n_pix = r.n_islands = r.n_lowgain = 0;
  r.flags = RTA_FLAG_BAD_DESCRIPTOR | RTA_FLAG_HILLAS_INVALID | RTA_FLAG_TIME_INVALID;
  *out = r;
}

// Waves per SIMD the register allocation must leave room for: the neighbour
// peak's 256-thread workgroups fit four to a compute unit by their LDS, if
// the registers allow it.  Elsewhere the compiler's own choice stands.
template <int EX, int NT>
constexpr int min_waves() {
  return EX == kExNeighbour && NT == 256 ? 4 : 1;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Unfused calibration: one workgroup per camera event, per-pixel results to HBM.
template <int EX, int PPL, int W, int NT>
__global__ __launch_bounds__(NT) void k_calibrate(DevCam c, const uint16_t* __restrict__ traces, int32_t* S,
                                                  int32_t* D, uint8_t* sstar, uint8_t* peak, uint8_t* gain,
                                                  float* q, float* t) {
  __shared__ uint32_t rows[EX == kExGlobal ? NT / kWave * 256 : (EX == kExNeighbour ? kMaxPix : 1)];
  __shared__ __attribute__((aligned(16))) uint16_t xrow[EX == kExNeighbour ? kNbrRows * (kMaxPix + 8) : 8];
  __shared__ int32_t start;
  const int64_t e = blockIdx.x;
  const int N = c.n_pix, np = c.n_pix_pad, T = c.n_samp;
  const uint16_t* ev = traces + e * c.event_elems;
  const size_t ob = (size_t)e * N;
  const __amdgpu_buffer_rsrc_t r = event_rsrc(ev, c.event_elems);
  if constexpr (EX == kExSliding && W == 4) {
    // the trace is read once: every pixel's window kept while it streams.
    // Pixels are independent here, so the pixel passes of an event are
    // spread over blockIdx.y: many more, shorter workgroups than events,
    // which evens out the last round of workgroups on a small batch
    const int npass = (N + NT * PPL - 1) / (NT * PPL);
    for (int ps = (int)blockIdx.y; ps < npass; ps += (int)gridDim.y) {
      const int pix0 = (ps * NT + (int)threadIdx.x) * PPL;
      KeepState<PPL> st;
      const uint32_t sw = keep_group<PPL, 2 * W>(c, r, pix0, np, T, c.n_gain == 2, st);
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        const int i = pix0 + p;
        if (i >= N) break;
        const int g = (sw >> p) & 1;
        const int s = 255 - (int)(st.key[p] & 255u);
        const int32_t P = c.P256[g * np + i];
        const int32_t d = key_to_d<W>(st.key[p], P);
        int pk;
        const int32_t nt = kept_nt(st.sv0[p], st.sv1[p], P, s, &pk);
        if (S) S[ob + i] = (int32_t)(st.key[p] >> 8);
        if (D) D[ob + i] = d;
        if (sstar) sstar[ob + i] = (uint8_t)s;
        if (peak) peak[ob + i] = (uint8_t)pk;
        if (gain) gain[ob + i] = (uint8_t)g;
        if (q) q[ob + i] = (float)d / (256.0f * c.a[g * np + i]);
        if (t) t[ob + i] = (float)peak_time<W>(s, nt, d);
      }
    }
    return;
  }
  extract_event<EX, PPL, W, 2 * W, NT>(c, r, ev, rows, &start, xrow, [&](int pix0, const uint32_t (&key)[PPL],
                                                                         uint32_t sw) {
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const int i = pix0 + p;
      if (i >= N) break;
      const int g = (sw >> p) & 1u;
      const int s = 255 - (int)(key[p] & 255u);
      const int32_t P = c.P256[g * np + i];
      const int32_t d = key_to_d<W>(key[p], P);
      int pk;
      const int32_t nt = window_nt<W>(ev + (size_t)g * T * np + i, np, s, P, &pk);
      const float tv = (float)peak_time<W>(s, nt, d);
      if (S) S[ob + i] = (int32_t)(key[p] >> 8);
      if (D) D[ob + i] = d;
      if (sstar) sstar[ob + i] = (uint8_t)s;
      if (peak) peak[ob + i] = (uint8_t)pk;
      if (gain) gain[ob + i] = (uint8_t)g;
      if (q) q[ob + i] = (float)d / (256.0f * c.a[g * np + i]);
      if (t) t[ob + i] = tv;
    }
  });
}

template <int NT>
__global__ __launch_bounds__(NT) void k_clean(DevCam c, const int32_t* __restrict__ D, const uint8_t* __restrict__ gain,
                                              uint8_t* __restrict__ mask, int have_levels, float t_pic, float t_bnd) {
  __shared__ TelSmem sm;
  const int64_t e = blockIdx.x;
  const int N = c.n_pix;
  const size_t ob = (size_t)e * N;
  for (int i = threadIdx.x; i < N; i += NT) {
    const int g = gain ? (int)gain[ob + i] : 0;
    sm.flag[i] = (uint8_t)(have_levels ? pixel_flag_at(c, g, i, D[ob + i], t_pic, t_bnd)
                                       : pixel_flag(c, g, i, D[ob + i]));
  }
  __syncthreads();
  mask_phase<NT>(c, sm);
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += NT) mask[ob + i] = (uint8_t)mask_bit(sm, i);
}

template <int W, int NT>
__global__ __launch_bounds__(NT) void k_hillas(DevCam c, const float* __restrict__ q, const int32_t* __restrict__ D,
                                               const float* __restrict__ t, const uint8_t* __restrict__ mask,
                                               const uint8_t* __restrict__ gain, rta_hillas_rec* out) {
  __shared__ TelSmem sm;
  const int64_t e = blockIdx.x;
  const int N = c.n_pix, nw = (N + 63) >> 6;
  const size_t ob = (size_t)e * N;
  const int lane = threadIdx.x & (kWave - 1);
  int nlow = 0;
  for (int base = threadIdx.x & ~(kWave - 1); base < nw * kWave; base += NT) {
    const int i = base + lane;
    const bool m = i < N && mask[ob + i] != 0;
    if (i < N && gain) nlow += gain[ob + i] == 1;
    const uint64_t b = __ballot(m);
    if (lane == 0) sm.mbits[base >> 6] = b;
  }
  post_count(sm, nlow);
  __syncthreads();
  scan_phase(N, sm);
  __syncthreads();
  const int n = sm.wbase[nw];
  list_phase<NT, W, false>(c, sm, nullptr, q ? q + ob : nullptr, D ? D + ob : nullptr, gain ? gain + ob : nullptr,
                           t + ob);
  __syncthreads();
  const rta_hillas_rec r = islands_hillas<NT, W, false>(c, sm, n, total_count<NT>(sm));
  if (threadIdx.x == 0) out[e] = r;
}

__global__ void k_queue_reset(unsigned long long* q) {
  if (threadIdx.x == 0) *q = 0ull;
}

// Classification of one telescope right after its Hillas parameters, by the
// first wavefront: the record is row 0 of a 16-row network tile (the other
// rows zero; a tile's rows do not affect each other, so the outputs equal
// those of the same record in any other tile), then the network-or-box-cut
// decision.  Lane 0 writes the score and log10 E and marks the fallback in
// the record; records without a valid image get NaN.  (Spreading the four
// tiles of each layer over four wavefronts, with the activations exchanged
// through LDS, was no faster: the layers wait on their weight loads.)
__device__ __forceinline__ void classify_telescope(const FusedArgs& a, long long tel, rta_hillas_rec& r) {
  const int lane = threadIdx.x & (kWave - 1), col = lane & 15, grp = lane >> 4;
  const bool valid = !(r.flags & RTA_FLAG_HILLAS_INVALID);
  float logit = 0.f, me = 0.f;
  if (valid && a.have_mlp) {  // uniform over the wavefront
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (col == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int f = 4 * grp + j;
        if (f < mlpdev::kIn) {
          const float z = (mlpdev::record_feature(r, f) - a.mlp.mean[f]) / a.mlp.stdv[f];
          v[j] = isfinite(z) ? z : 0.f;
        }
      }
    }
    mlpdev::bf16x4 h1[4], h2[4], h3[4];
    const mlpdev::f32x4 o = mlpdev::mlp_forward_tile(a.mlp, mlpdev::pack4(v[0], v[1], v[2], v[3]), h1, h2, h3);
    logit = o[0];
    me = o[1];
  }
  if (lane == 0) {
    float score = kNaN, log10e = kNaN;
    if (valid) {
      const mlpdev::ClassOut co = mlpdev::classify_record(r, a.bc, a.have_mlp != 0, logit, me);
      if (co.fallback) r.flags |= RTA_FLAG_MLP_FALLBACK;
      score = co.score;
      log10e = co.log10e;
    }
    a.tel_class[2 * tel] = score;
    a.tel_class[2 * tel + 1] = log10e;
  }
}

// Per-telescope body of the fused kernel: descriptor checks, then
// calibration -> cleaning -> Hillas with all intermediates in LDS.
template <int EX, int PPL, int W, int CH, int NT>
__device__ __forceinline__ void fused_telescope(const FusedArgs& a, long long tel, TelSmem& sm) {
  const int ty = uniform_i32(a.tel_type[tel]);
  const long long off = uniform_i64(a.tel_trace_off[tel]);
  const uint32_t bad = tel_descriptor_status(ty, off, a.n_types, a.traces_len,
                                             [&](int t) { return (int64_t)a.cams[t].event_elems; });
  if (bad) {
    if (threadIdx.x == 0) {
      bad_record(a.out + tel);
      if (a.classify) {
        a.tel_class[2 * tel] = kNaN;
        a.tel_class[2 * tel + 1] = kNaN;
      }
      atomicOr(a.status, bad);
    }
    return;
  }
  rta_hillas_rec r = process_telescope<EX, PPL, W, CH, NT>(a.cams[ty], uniform_ptr(a.traces + off), sm);
  if (a.classify && threadIdx.x < kWave) classify_telescope(a, tel, r);
  if (threadIdx.x == 0) a.out[tel] = r;
}

// Persistent form: a fixed grid of workgroups pulls telescopes from a global
// counter until the batch is drained.
template <int EX, int PPL, int W, int CH, int NT>
__global__ __launch_bounds__(NT) void k_fused(FusedArgs a) {
  __shared__ TelSmem sm;
  __shared__ long long s_tel;
  for (;;) {
    if (threadIdx.x == 0) s_tel = (long long)atomicAdd(a.queue, 1ull);
    __syncthreads();
    const long long tel = uniform_i64(s_tel);
    __syncthreads();
    if (tel >= a.n_tel) return;
    fused_telescope<EX, PPL, W, CH, NT>(a, tel, sm);
    __syncthreads();
  }
}

// Grid form: one workgroup per telescope, dispatched by the hardware's
// workgroup scheduler (no loop-carried state, so no register pressure from
// values hoisted across telescopes).
template <int EX, int PPL, int W, int CH, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(min_waves<EX, NT>()))) void k_fused_grid(
    FusedArgs a) {
  __shared__ TelSmem sm;
  fused_telescope<EX, PPL, W, CH, NT>(a, (long long)blockIdx.x, sm);
}

// One wavefront per array event: stereo direction from the telescope records
// and, when enabled, per-telescope classification (network on 16-telescope
// MFMA tiles, box-cut fallback) aggregated into size-weighted event values.
constexpr int kEvtNT = 256;
__global__ __launch_bounds__(kEvtNT) void k_event(EventArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t e = (int64_t)blockIdx.x * (kEvtNT / kWave) + (threadIdx.x / kWave);
  if (e >= a.n_evt) return;
  const int64_t lo = a.evt_tel_off[e], hi = a.evt_tel_off[e + 1];
  rta_event_rec r;
  r.gammaness = kNaN;
  r.log10_energy = kNaN;
  if (!event_range_ok(lo, hi, a.n_tel)) {
    if (lane == 0) {
      r.dir_x = r.dir_y = r.cond = kNaN;
      r.n_tel = 0;
      r.n_used = 0;
      r.flags = RTA_EVT_STEREO_INVALID | RTA_EVT_NO_MLP;
      a.out[e] = r;
      if (a.done_clock) a.done_clock[e] = wall_clock64();
      atomicOr(a.status, RTA_STATUS_BAD_EVENT);
    }
    return;
  }
  float v[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // A00, A01, A11, b0, b1, used
  for (int64_t k = lo + lane; k < hi; k += kWave) {
    const int ty = a.tel_type[k];
    if (ty < 0 || ty >= a.n_types) continue;
    const rta_hillas_rec h = a.tel[k];
    if (h.flags & (RTA_FLAG_HILLAS_INVALID | RTA_FLAG_BAD_DESCRIPTOR)) continue;
    if (!(h.length > 0.f) || !(h.width >= 0.f) || !isfinite(h.psi) || !isfinite(h.size)) continue;
    const float ratio = h.width / h.length;
    if (ratio > a.max_width_ratio) continue;
    const float w = h.size * (1.0f - ratio);
    const float f = a.focal[ty];
    const float nx = -sinf(h.psi), ny = cosf(h.psi);
    const float cx = h.cog_x / f, cy = h.cog_y / f;
    const float nc = nx * cx + ny * cy;
    v[0] += w * nx * nx;
    v[1] += w * nx * ny;
    v[2] += w * ny * ny;
    v[3] += w * nc * nx;
    v[4] += w * nc * ny;
    v[5] += 1.f;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
#pragma unroll
    for (int off = kWave / 2; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, kWave);
  }
  // classification: rows = telescopes of this event, 16 per MFMA tile
  float c[3] = {0.f, 0.f, 0.f};  // sum size*score, sum size*log10E, sum size
  if (a.have_box) {
    const int col = lane & 15, grp = lane >> 4;
    for (int64_t r0 = lo; r0 < hi; r0 += 16) {
      float logit = 0.f, me = 0.f;
      if (a.have_mlp && !a.tel_class) {
        mlpdev::bf16x4 h1[4], h2[4], h3[4];
        const mlpdev::bf16x4 xin = mlpdev::mlp_record_tile(a.mlp, a.tel, hi, r0);
        const mlpdev::f32x4 o = mlpdev::mlp_forward_tile(a.mlp, xin, h1, h2, h3);
        logit = o[0];
        me = o[1];
      }
      const int64_t k = r0 + col;
      if (grp == 0 && k < hi) {
        rta_hillas_rec h = a.tel[k];
        const int ty = a.tel_type[k];
        if (ty >= 0 && ty < a.n_types && !(h.flags & (RTA_FLAG_HILLAS_INVALID | RTA_FLAG_BAD_DESCRIPTOR))) {
          float score, log10e;
          if (a.tel_class) {  // classified in the reconstruction kernel
            score = a.tel_class[2 * k];
            log10e = a.tel_class[2 * k + 1];
          } else {
            const mlpdev::ClassOut co = mlpdev::classify_record(h, a.bc, a.have_mlp != 0, logit, me);
            if (co.fallback) a.tel[k].flags = h.flags | RTA_FLAG_MLP_FALLBACK;
            score = co.score;
            log10e = co.log10e;
          }
          if (isfinite(log10e) && h.size > 0.f) {
            c[0] += h.size * score;
            c[1] += h.size * log10e;
            c[2] += h.size;
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int off = kWave / 2; off >= 1; off >>= 1) c[k] += __shfl_xor(c[k], off, kWave);
    }
  }
  if (lane == 0) {
    const float A00 = v[0], A01 = v[1], A11 = v[2], b0 = v[3], b1 = v[4];
    const float tr = A00 + A11, det = A00 * A11 - A01 * A01;
    const float hd = 0.5f * (A00 - A11);
    const float lmax = 0.5f * tr + sqrtf(hd * hd + A01 * A01);
    const float lmin = lmax > 0.f ? det / lmax : 0.f;
    const float cond = lmin > 0.f ? lmax / lmin : INFINITY;
    r.cond = cond;
    r.n_tel = (int32_t)(hi - lo);
    r.n_used = (int32_t)v[5];
    r.flags = a.have_mlp ? 0u : RTA_EVT_NO_MLP;
    if (r.n_used < 2 || !(cond < a.max_cond)) {
      r.dir_x = r.dir_y = kNaN;
      r.flags |= RTA_EVT_STEREO_INVALID;
    } else {
      r.dir_x = (A11 * b0 - A01 * b1) / det;
      r.dir_y = (A00 * b1 - A01 * b0) / det;
    }
    if (a.have_box && c[2] > 0.f) {
      r.gammaness = c[0] / c[2];
      r.log10_energy = c[1] / c[2];
    }
    a.out[e] = r;
    if (a.done_clock) a.done_clock[e] = wall_clock64();
  }
}

__global__ void k_stamp(uint64_t* slot) {
  if (threadIdx.x == 0) *slot = wall_clock64();
}

// Network inputs of records, one thread per record.
__global__ __launch_bounds__(256) void k_features(const rta_hillas_rec* __restrict__ rec, int64_t n,
                                                  float* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const rta_hillas_rec r = rec[i];
#pragma unroll
  for (int f = 0; f < mlpdev::kIn; ++f) x[i * mlpdev::kIn + f] = mlpdev::record_feature(r, f);
}

// Per-record classification, one wavefront per 16 records.
__global__ __launch_bounds__(256) void k_classify(MlpDev w, int have_mlp, rta_boxcut_desc bc,
                                                  const rta_hillas_rec* __restrict__ rec, int64_t n,
                                                  float* __restrict__ out) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (r0 >= n) return;
  float logit = 0.f, me = 0.f;
  if (have_mlp) {
    mlpdev::bf16x4 h1[4], h2[4], h3[4];
    const mlpdev::f32x4 o = mlpdev::mlp_forward_tile(w, mlpdev::mlp_record_tile(w, rec, n, r0), h1, h2, h3);
    logit = o[0];
    me = o[1];
  }
  const int64_t k = r0 + col;
  if (grp == 0 && k < n) {
    const mlpdev::ClassOut co = mlpdev::classify_record(rec[k], bc, have_mlp != 0, logit, me);
    out[k * 4 + 0] = co.score;
    out[k * 4 + 1] = co.log10e;
    out[k * 4 + 2] = (float)co.gamma;
    out[k * 4 + 3] = (float)co.fallback;
  }
}

// ---------------------------------------------------------------------------
// Dispatch tables
// ---------------------------------------------------------------------------
constexpr int kUnfusedNT = 256;
constexpr int kUnfusedPPL = 4;
constexpr int kKeepPPL = 2;  // sliding-window calibrate: the kept windows take registers

template <int W>
hipError_t launch_calibrate_w(const DevCam& c, int ex, const uint16_t* tr, int64_t n, int32_t* S, int32_t* D,
                              uint8_t* ss, uint8_t* pk, uint8_t* g, float* q, float* t, hipStream_t st) {
  switch (ex) {
    case kExSliding: {
      const unsigned npass = (unsigned)((c.n_pix + kUnfusedNT * kKeepPPL - 1) / (kUnfusedNT * kKeepPPL));
      hipLaunchKernelGGL((k_calibrate<kExSliding, kKeepPPL, W, kUnfusedNT>), dim3((unsigned)n, npass),
                         dim3(kUnfusedNT), 0, st, c, tr, S, D, ss, pk, g, q, t);
      break;
    }
    case kExFixed:
      hipLaunchKernelGGL((k_calibrate<kExFixed, kUnfusedPPL, W, kUnfusedNT>), dim3((unsigned)n), dim3(kUnfusedNT), 0,
                         st, c, tr, S, D, ss, pk, g, q, t);
      break;
    case kExGlobal:
      hipLaunchKernelGGL((k_calibrate<kExGlobal, kUnfusedPPL, W, kUnfusedNT>), dim3((unsigned)n), dim3(kUnfusedNT),
                         0, st, c, tr, S, D, ss, pk, g, q, t);
      break;
    case kExNeighbour:
      hipLaunchKernelGGL((k_calibrate<kExNeighbour, kUnfusedPPL, W, kUnfusedNT>), dim3((unsigned)n),
                         dim3(kUnfusedNT), 0, st, c, tr, S, D, ss, pk, g, q, t);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W>
hipError_t launch_hillas_w(const DevCam& c, const float* q, const int32_t* D, const float* t, const uint8_t* m,
                           const uint8_t* g, int64_t n, rta_hillas_rec* out, hipStream_t st) {
  hipLaunchKernelGGL((k_hillas<W, kUnfusedNT>), dim3((unsigned)n), dim3(kUnfusedNT), 0, st, c, q, D, t, m, g, out);
  return hipGetLastError();
}

// grid == 0: one workgroup per telescope; otherwise the persistent form
// (sliding window only: the other extractors always use the grid form).
template <int PPL, int W, int CH, int NT>
hipError_t launch_fused_t(const FusedArgs& a, int grid, hipStream_t st) {
  const dim3 g1((unsigned)a.n_tel);
  switch (a.extractor) {
    case kExSliding:
      if (grid == 0)
        hipLaunchKernelGGL((k_fused_grid<kExSliding, PPL, W, CH, NT>), g1, dim3(NT), 0, st, a);
      else
        hipLaunchKernelGGL((k_fused<kExSliding, PPL, W, CH, NT>), dim3(grid), dim3(NT), 0, st, a);
      break;
    case kExFixed: hipLaunchKernelGGL((k_fused_grid<kExFixed, PPL, W, CH, NT>), g1, dim3(NT), 0, st, a); break;
    case kExGlobal: hipLaunchKernelGGL((k_fused_grid<kExGlobal, PPL, W, CH, NT>), g1, dim3(NT), 0, st, a); break;
    case kExNeighbour:
      hipLaunchKernelGGL((k_fused_grid<kExNeighbour, PPL, W, CH, NT>), g1, dim3(NT), 0, st, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W>
hipError_t launch_fused_w(const FusedArgs& a, const rta_schedule& s, int grid, hipStream_t st) {
  const int key = s.pix_per_lane * 1000 + s.waves_per_wg * 100 + s.chunk;
  switch (key) {
    case 2408: return launch_fused_t<2, W, 8, 256>(a, grid, st);
    case 2416: return launch_fused_t<2, W, 16, 256>(a, grid, st);
    case 2808: return launch_fused_t<2, W, 8, 512>(a, grid, st);
    case 2816: return launch_fused_t<2, W, 16, 512>(a, grid, st);
    case 4408: return launch_fused_t<4, W, 8, 256>(a, grid, st);
    case 4416: return launch_fused_t<4, W, 16, 256>(a, grid, st);
    case 4808: return launch_fused_t<4, W, 8, 512>(a, grid, st);
    case 4816: return launch_fused_t<4, W, 16, 512>(a, grid, st);
    case 8408: return launch_fused_t<8, W, 8, 256>(a, grid, st);
    case 8416: return launch_fused_t<8, W, 16, 256>(a, grid, st);
    case 8808: return launch_fused_t<8, W, 8, 512>(a, grid, st);
    case 8816: return launch_fused_t<8, W, 16, 512>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool window_supported(int w) { return w == 4; }

bool extractor_supported(int ex) {
  return ex == kExSliding || ex == kExFixed || ex == kExGlobal || ex == kExNeighbour;
}

bool schedule_supported(const rta_schedule& s) {
  const bool ppl = s.pix_per_lane == 2 || s.pix_per_lane == 4 || s.pix_per_lane == 8;
  const bool wv = s.waves_per_wg == 4 || s.waves_per_wg == 8;
  const bool ch = s.chunk == 8 || s.chunk == 16;
  return ppl && wv && ch && s.wg_per_cu >= 0 && s.wg_per_cu <= 4;
}

int list_schedules(rta_schedule* out, int cap) {
  int n = 0;
  const int ppls[3] = {2, 4, 8}, waves[2] = {4, 8}, chunks[2] = {8, 16};
  for (int p : ppls)
    for (int w : waves)
      for (int ch : chunks)
        for (int g = 0; g <= 4; ++g) {
          if (out && n < cap) out[n] = rta_schedule{p, w, g, ch};
          ++n;
        }
  return n;
}

hipError_t launch_calibrate(const DevCam& c, int extractor, const uint16_t* traces, int64_t n_evt, int32_t* S,
                            int32_t* D, uint8_t* sstar, uint8_t* peak, uint8_t* gain, float* q, float* t,
                            hipStream_t st) {
  switch (c.window) {
    case 4: return launch_calibrate_w<4>(c, extractor, traces, n_evt, S, D, sstar, peak, gain, q, t, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_clean(const DevCam& c, const rta_clean_params* levels, const int32_t* D, const uint8_t* gain,
                        int64_t n_evt, uint8_t* mask, hipStream_t st) {
  hipLaunchKernelGGL((k_clean<kUnfusedNT>), dim3((unsigned)n_evt), dim3(kUnfusedNT), 0, st, c, D, gain, mask,
                     levels ? 1 : 0, levels ? levels->t_pic : 0.f, levels ? levels->t_bnd : 0.f);
  return hipGetLastError();
}

hipError_t launch_hillas(const DevCam& c, const float* q, const int32_t* D, const float* t, const uint8_t* mask,
                         const uint8_t* gain, int64_t n_evt, rta_hillas_rec* out, hipStream_t st) {
  switch (c.window) {
    case 4: return launch_hillas_w<4>(c, q, D, t, mask, gain, n_evt, out, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_queue_reset(unsigned long long* queue, hipStream_t st) {
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, st, queue);
  return hipGetLastError();
}

hipError_t launch_fused(const FusedArgs& a, const rta_schedule& s, int n_cu, hipStream_t st) {
  long long grid = (long long)n_cu * s.wg_per_cu;
  if (grid > a.n_tel) grid = a.n_tel;
  if (grid < 1) grid = 1;
  if (s.wg_per_cu == 0 || a.extractor != kExSliding) grid = 0;
  switch (a.window) {
    case 4: return launch_fused_w<4>(a, s, (int)grid, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_features(const rta_hillas_rec* rec, int64_t n, float* x, hipStream_t st) {
  hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rec, n, x);
  return hipGetLastError();
}

hipError_t launch_classify(const MlpDev& w, bool have_mlp, const rta_boxcut_desc& bc, const rta_hillas_rec* rec,
                           int64_t n, float* out, hipStream_t st) {
  const int64_t tiles = (n + 15) / 16;
  hipLaunchKernelGGL(k_classify, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, w, have_mlp ? 1 : 0, bc, rec, n,
                     out);
  return hipGetLastError();
}

hipError_t launch_stamp(uint64_t* slot, hipStream_t st) {
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, st, slot);
  return hipGetLastError();
}

hipError_t launch_event(const EventArgs& a, hipStream_t st) {
  const int64_t per = kEvtNT / kWave;
  const int64_t grid = (a.n_evt + per - 1) / per;
  hipLaunchKernelGGL(k_event, dim3((unsigned)grid), dim3(kEvtNT), 0, st, a);
  return hipGetLastError();
}

}  // namespace rta
