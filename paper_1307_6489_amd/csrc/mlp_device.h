// Device building blocks of the BF16-MFMA network, shared by the training
// kernels (mlp.hip) and the per-array-event kernel (reco.hip).
#pragma once

#include "rta_internal.h"

namespace rta {
namespace mlpdev {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 10, kHid = 64, kOut = 2;
constexpr int kInPad = 16, kOutPad = 16;


// float -> bfloat16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  bf16x4 v;
  v[0] = (short)f2bf(a);
  v[1] = (short)f2bf(b);
  v[2] = (short)f2bf(c);
  v[3] = (short)f2bf(d);
  return v;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// One 16x16 tile product over K = 16 (v_mfma_f32_16x16x16_bf16).
__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// One 16x16 tile product over two K = 16 blocks at once
// (v_mfma_f32_16x16x32_bf16): lane group g supplies eight k slots, the
// four of block 0 then the four of block 1 that the K = 16 layout gives it.
// Both operands use the same slot order, so the contraction is the sum over
// both blocks whatever k each slot stands for.
__device__ __forceinline__ f32x4 mfma2(bf16x4 a0, bf16x4 a1, bf16x4 b0, bf16x4 b1, f32x4 c) {
  const bf16x8 a = __builtin_bit_cast(bf16x8, __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7));
  const bf16x8 b = __builtin_bit_cast(bf16x8, __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7));
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// A operand: 4 consecutive bf16 of row `row` starting at column `col0`.
__device__ __forceinline__ bf16x4 load4(const uint16_t* M, int ld, int row, int col0) {
  return *reinterpret_cast<const bf16x4*>(M + (size_t)row * ld + col0);
}

__device__ __forceinline__ f32x4 bias4(const float* b, int o) {
  f32x4 v;
  v[0] = b[o]; v[1] = b[o + 1]; v[2] = b[o + 2]; v[3] = b[o + 3];
  return v;
}

__device__ __forceinline__ bf16x4 relu_bf(f32x4 a) {
  return pack4(fmaxf(a[0], 0.f), fmaxf(a[1], 0.f), fmaxf(a[2], 0.f), fmaxf(a[3], 0.f));
}

// g * [h > 0] elementwise, rounded to bf16 (h is a ReLU output, >= 0).
__device__ __forceinline__ bf16x4 mask_bf(f32x4 g, bf16x4 h) {
  return pack4(h[0] ? g[0] : 0.f, h[1] ? g[1] : 0.f, h[2] ? g[2] : 0.f, h[3] ? g[3] : 0.f);
}

__device__ __forceinline__ void store4T(uint16_t* MT, int ldb, int f0, int b, bf16x4 v) {
  MT[(size_t)(f0 + 0) * ldb + b] = (uint16_t)v[0];
  MT[(size_t)(f0 + 1) * ldb + b] = (uint16_t)v[1];
  MT[(size_t)(f0 + 2) * ldb + b] = (uint16_t)v[2];
  MT[(size_t)(f0 + 3) * ldb + b] = (uint16_t)v[3];
}

// Forward of one 16-row tile by one wavefront.  xin: B-operand tile of the
// standardised inputs (lane: row l%16, features 4*(l/16)..+3).  Returns the
// output accumulator (lanes 0..15: [logit, log10 E, 0, 0] of row l%16) and
// the three hidden activations in B-operand layout.
__device__ __forceinline__ f32x4 mlp_forward_tile(const MlpDev& w, bf16x4 xin, bf16x4 (&h1)[4], bf16x4 (&h2)[4],
                                                  bf16x4 (&h3)[4]) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = bias4(w.b1, 16 * t + 4 * grp);
    acc = mfma(load4(w.W1t, kInPad, 16 * t + col, 4 * grp), xin, acc);
    h1[t] = relu_bf(acc);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = bias4(w.b2, 16 * t + 4 * grp);
#pragma unroll
    for (int u = 0; u < 4; u += 2)
      acc = mfma2(load4(w.W2t, kHid, 16 * t + col, 16 * u + 4 * grp),
                  load4(w.W2t, kHid, 16 * t + col, 16 * (u + 1) + 4 * grp), h1[u], h1[u + 1], acc);
    h2[t] = relu_bf(acc);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = bias4(w.b3, 16 * t + 4 * grp);
#pragma unroll
    for (int u = 0; u < 4; u += 2)
      acc = mfma2(load4(w.W3t, kHid, 16 * t + col, 16 * u + 4 * grp),
                  load4(w.W3t, kHid, 16 * t + col, 16 * (u + 1) + 4 * grp), h2[u], h2[u + 1], acc);
    h3[t] = relu_bf(acc);
  }
  f32x4 out = bias4(w.b4, 4 * grp);
#pragma unroll
  for (int u = 0; u < 4; u += 2)
    out = mfma2(load4(w.W4t, kHid, col, 16 * u + 4 * grp), load4(w.W4t, kHid, col, 16 * (u + 1) + 4 * grp), h3[u],
                h3[u + 1], out);
  return out;
}

// Standardised input tile of rows r0..r0+15 (row-major raw features [B][10]).
__device__ __forceinline__ bf16x4 mlp_input_tile(const MlpDev& w, const float* x, int B, int r0) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  const int b = r0 + col;
  float v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int f = 4 * grp + j;
    v[j] = (b < B && f < kIn) ? (x[(size_t)b * kIn + f] - w.mean[f]) / w.stdv[f] : 0.f;
  }
  return pack4(v[0], v[1], v[2], v[3]);
}

// The 10 network inputs of a Hillas record.
__device__ __forceinline__ float record_feature(const rta_hillas_rec& r, int f) {
  switch (f) {
    case 0: return log10f(r.size);
    case 1: return r.length;
    case 2: return r.width;
    case 3: return r.cog_dist;
    case 4: return r.psi;
    case 5: return r.skewness;
    case 6: return r.kurtosis;
    case 7: return r.time_gradient;
    case 8: return r.leakage;
    default: return (float)r.n_islands;
  }
}

// Standardised input tile from records rec[r0 .. r0+15] (rows >= n are 0).
__device__ __forceinline__ bf16x4 mlp_record_tile(const MlpDev& w, const rta_hillas_rec* rec, int64_t n, int64_t r0) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  if (r0 + col < n) {
    const rta_hillas_rec r = rec[r0 + col];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int f = 4 * grp + j;
      if (f < kIn) {
        const float z = (record_feature(r, f) - w.mean[f]) / w.stdv[f];
        v[j] = isfinite(z) ? z : 0.f;  // non-finite rows fall back to the box cuts
      }
    }
  }
  return pack4(v[0], v[1], v[2], v[3]);
}

struct ClassOut {
  float score, log10e;
  int gamma, fallback;
};

// Decision for one record given the network outputs (have_mlp) and the
// box-cut tables.  The network is used when every feature is finite and
// inside the trained range; otherwise the box cuts decide.
__device__ __forceinline__ ClassOut classify_record(const rta_hillas_rec& r, const rta_boxcut_desc& bc, bool have_mlp,
                                                    float logit, float mlp_e) {
  ClassOut o;
  bool in_range = have_mlp;
#pragma unroll
  for (int f = 0; f < kIn; ++f) {
    const float v = record_feature(r, f);
    in_range = in_range && isfinite(v) && v >= bc.feat_lo[f] && v <= bc.feat_hi[f];
  }
  const float lgs = log10f(r.size);
  if (in_range) {
    o.score = 1.f / (1.f + expf(-logit));
    o.log10e = mlp_e;
    o.gamma = o.score > bc.mlp_cut;
    o.fallback = 0;
  } else {
    int b = (int)floorf((lgs - bc.lgs_lo) / (bc.lgs_hi - bc.lgs_lo) * (float)bc.n_bins);
    b = b < 0 ? 0 : (b >= bc.n_bins ? bc.n_bins - 1 : b);
    const float sw = (r.width - bc.w_mean[b]) / bc.w_std[b];
    const float sl = (r.length - bc.l_mean[b]) / bc.l_std[b];
    o.gamma = (sw < bc.cut_w) && (sl < bc.cut_l);
    o.score = o.gamma ? 1.f : 0.f;
    o.log10e = bc.e_a + bc.e_b * lgs;
    o.fallback = 1;
  }
  return o;
}

}  // namespace mlpdev
}  // namespace rta
