// Gamma/hadron + energy network on BF16 matrix cores (gfx950 MFMA).
//
// The network (10 -> 64 -> 64 -> 64 -> 2, ReLU) maps per-telescope image
// parameters to a gamma logit and log10(E/TeV); it fills the gamma/hadron
// separation and energy steps that the paper lists among the reconstruction
// products (Section 4.1).  Operands are bfloat16, accumulation FP32.
//
// Register layout.  Every layer is computed transposed, Z^T = W^T . H^T, on
// 16x16 tiles: A = a block of W^T (rows = output features), B = a block of
// H^T (features x 16 rows), C/D = 16 output features x 16 rows.  In that
// orientation the accumulator layout (lane l: row-of-batch l%16, features
// 4*(l/16)..+3) is exactly the B-operand layout of a 16-feature block, so
// activations go from one layer to the next in registers.  Contractions over
// 64 features (or over the batch) take two 16-blocks per
// v_mfma_f32_16x16x32_bf16, the two blocks' B fragments side by side; the
// 16-wide input and output layers use v_mfma_f32_16x16x16_bf16.
// The backward pass uses the same trick with the untransposed weights.  Weight
// gradients contract over the batch, so per-row activations and gradients are
// written feature-major ([F][B], bf16) and wavefronts, one per 16x16 weight
// tile and batch slice, run the batch contraction with the same instruction.
#include <cmath>

#include "mlp_device.h"
#include "mlp_launch.h"

namespace rta {
using namespace mlpdev;
constexpr int kRowsNT = 256;  // 4 wavefronts, 16 rows each

namespace {

// Standardised input tile of batch rows r0..r0+15 taken from data rows
// rows[b] (clamped to [0, n_data)) of x [n_data][10].
__device__ __forceinline__ bf16x4 gather_input_tile(const MlpDev& w, const float* x, const int64_t* rows,
                                                    int64_t n_data, int B, int r0) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  const int b = r0 + col;
  int64_t d = 0;
  if (b < B) d = min(max(rows[b], (int64_t)0), n_data - 1);
  float v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int f = 4 * grp + j;
    v[j] = (b < B && f < kIn) ? (x[d * kIn + f] - w.mean[f]) / w.stdv[f] : 0.f;
  }
  return pack4(v[0], v[1], v[2], v[3]);
}

// Forward (+ loss, + backward to every layer's pre-activation gradient when
// TRAIN) of 16-row tiles, one per wavefront.  rows != null: batch row b is
// data row rows[b] of x / label / log10e (the batch gather done here
// instead of in separate copies).
template <bool TRAIN>
__global__ __launch_bounds__(kRowsNT) void k_mlp_rows(MlpDev w, const float* __restrict__ x,
                                                      const float* __restrict__ label,
                                                      const float* __restrict__ log10e,
                                                      const int64_t* __restrict__ rows, int64_t n_data, int B,
                                                      int Bpad, float* __restrict__ out) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  const int r0 = (blockIdx.x * (kRowsNT / 64) + (threadIdx.x >> 6)) * 16;
  if (r0 >= Bpad) return;
  const int b = r0 + col;
  const bool valid = b < B;
  const bf16x4 xin = rows ? gather_input_tile(w, x, rows, n_data, B, r0) : mlp_input_tile(w, x, B, r0);
  const int64_t db = (rows && valid) ? min(max(rows[b], (int64_t)0), n_data - 1) : (int64_t)b;
  bf16x4 h1[4], h2[4], h3[4];
  const f32x4 o = mlp_forward_tile(w, xin, h1, h2, h3);
  if (!TRAIN) {
    if (grp == 0 && valid) {
      out[(size_t)b * 2] = o[0];
      out[(size_t)b * 2 + 1] = o[1];
    }
    return;
  }
  // loss and output gradient (lanes of group 0 own the two outputs of row b)
  float g0 = 0.f, g1 = 0.f;
  if (grp == 0) {
    float lrow = 0.f;
    if (valid) {
      const float z = o[0], e = o[1], lab = label[db], y = log10e[db];
      const float m = lab > 0.5f ? 1.f : 0.f;
      const float sig = 1.f / (1.f + expf(-z));
      lrow = fmaxf(z, 0.f) - z * lab + log1pf(expf(-fabsf(z))) + m * (e - y) * (e - y);
      g0 = (sig - lab) / (float)B;
      g1 = 2.f * m * (e - y) / (float)B;
    }
    w.loss_row[b] = lrow;
  }
  const bf16x4 g4 = pack4(g0, g1, 0.f, 0.f);
  // store H^T and G4^T (feature-major) for the weight-gradient contraction
  store4T(w.H0, Bpad, 4 * grp, b, xin);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    store4T(w.H1, Bpad, 16 * t + 4 * grp, b, h1[t]);
    store4T(w.H2, Bpad, 16 * t + 4 * grp, b, h2[t]);
    store4T(w.H3, Bpad, 16 * t + 4 * grp, b, h3[t]);
  }
  store4T(w.G4, Bpad, 4 * grp, b, g4);
  // dH3^T = W4 . G4^T, masked -> G3; then G2, G1
  bf16x4 g3[4], g2[4], g1v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(load4(w.W4n, kOutPad, 16 * t + col, 4 * grp), g4, acc);
    g3[t] = mask_bf(acc, h3[t]);
    store4T(w.G3, Bpad, 16 * t + 4 * grp, b, g3[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 4; u += 2)
      acc = mfma2(load4(w.W3n, kHid, 16 * t + col, 16 * u + 4 * grp),
                  load4(w.W3n, kHid, 16 * t + col, 16 * (u + 1) + 4 * grp), g3[u], g3[u + 1], acc);
    g2[t] = mask_bf(acc, h2[t]);
    store4T(w.G2, Bpad, 16 * t + 4 * grp, b, g2[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 4; u += 2)
      acc = mfma2(load4(w.W2n, kHid, 16 * t + col, 16 * u + 4 * grp),
                  load4(w.W2n, kHid, 16 * t + col, 16 * (u + 1) + 4 * grp), g2[u], g2[u + 1], acc);
    g1v[t] = mask_bf(acc, h1[t]);
    store4T(w.G1, Bpad, 16 * t + 4 * grp, b, g1v[t]);
  }
}

// Weight / bias gradients and the loss.  The batch contraction of each 16x16
// weight tile (40) and bias vector (4) is cut into kGradSplit slices of
// consecutive 16-row blocks, one wavefront per (tile, slice), each writing
// its partial sums to gpart[slice]; a last wavefront sums the loss.  The
// slices are added in slice order by grad_sum (fixed order: the gradient is
// reproducible).  One long contraction per tile would leave the chip nearly
// idle and every step waiting on the previous load.
constexpr int kGradTiles = 44;
constexpr int kGradBlocks = kGradTiles * kGradSplit + 1;

__global__ __launch_bounds__(64) void k_mlp_grad(MlpDev w, int B, int Bpad, float* __restrict__ loss_out) {
  const int lane = threadIdx.x, col = lane & 15, grp = lane >> 4;
  if (blockIdx.x == kGradTiles * kGradSplit) {
    // 16 loads in flight per step, added in row order
    float s = 0.f;
    int r = lane;
    for (; r + 64 * 15 < B; r += 64 * 16) {
      float v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = w.loss_row[r + 64 * u];
#pragma unroll
      for (int u = 0; u < 16; ++u) s += v[u];
    }
    for (; r < B; r += 64) s += w.loss_row[r];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) {
      const float L = s / (float)B;
      if (loss_out) *loss_out = L;
      w.loss_row[Bpad] = L;
    }
    return;
  }
  const int wv = blockIdx.x / kGradSplit, sl = blockIdx.x % kGradSplit;
  const int nk = Bpad / 16, per = (nk + kGradSplit - 1) / kGradSplit;
  const int k0 = min(nk, sl * per), k1 = min(nk, k0 + per);
  float* __restrict__ part = w.gpart + (size_t)sl * kNParams;
  if (wv < 40) {
    // tile -> (layer, input chunk, output chunk)
    const uint16_t *H, *G;
    int in0, out0, in_dim, out_dim, off;
    if (wv < 4) { H = w.H0; G = w.G1; in0 = 0; out0 = 16 * wv; in_dim = kIn; out_dim = kHid; off = kOffW1; }
    else if (wv < 20) { const int t = wv - 4; H = w.H1; G = w.G2; in0 = 16 * (t / 4); out0 = 16 * (t % 4); in_dim = kHid; out_dim = kHid; off = kOffW2; }
    else if (wv < 36) { const int t = wv - 20; H = w.H2; G = w.G3; in0 = 16 * (t / 4); out0 = 16 * (t % 4); in_dim = kHid; out_dim = kHid; off = kOffW3; }
    else { H = w.H3; G = w.G4; in0 = 16 * (wv - 36); out0 = 0; in_dim = kHid; out_dim = kOut; off = kOffW4; }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    int k = k0;
    for (; k + 4 <= k1; k += 4) {  // four 16-row blocks loaded before their MFMAs
      bf16x4 a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = load4(H, Bpad, in0 + col, 16 * (k + u) + 4 * grp);
        b[u] = load4(G, Bpad, out0 + col, 16 * (k + u) + 4 * grp);
      }
#pragma unroll
      for (int u = 0; u < 4; u += 2) acc = mfma2(a[u], a[u + 1], b[u], b[u + 1], acc);
    }
    for (; k + 2 <= k1; k += 2)
      acc = mfma2(load4(H, Bpad, in0 + col, 16 * k + 4 * grp), load4(H, Bpad, in0 + col, 16 * (k + 1) + 4 * grp),
                  load4(G, Bpad, out0 + col, 16 * k + 4 * grp), load4(G, Bpad, out0 + col, 16 * (k + 1) + 4 * grp),
                  acc);
    if (k < k1)
      acc = mfma(load4(H, Bpad, in0 + col, 16 * k + 4 * grp), load4(G, Bpad, out0 + col, 16 * k + 4 * grp), acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = in0 + 4 * grp + i, n = out0 + col;
      if (m < in_dim && n < out_dim) part[off + m * out_dim + n] = acc[i];
    }
  } else {
    const int l = wv - 40;  // bias of layer l+1
    const uint16_t* G = l == 0 ? w.G1 : l == 1 ? w.G2 : l == 2 ? w.G3 : w.G4;
    const int nchunk = l == 3 ? 1 : 4, dim = l == 3 ? kOut : kHid;
    const int off = l == 0 ? kOffB1 : l == 1 ? kOffB2 : l == 2 ? kOffB3 : kOffB4;
    bf16x4 ones;
    ones[0] = ones[1] = ones[2] = ones[3] = (short)0x3F80;  // bf16(1.0)
    for (int c = 0; c < nchunk; ++c) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      int k = k0;
      for (; k + 4 <= k1; k += 4) {
        bf16x4 b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) b[u] = load4(G, Bpad, 16 * c + col, 16 * (k + u) + 4 * grp);
#pragma unroll
        for (int u = 0; u < 4; u += 2) acc = mfma2(ones, ones, b[u], b[u + 1], acc);
      }
      for (; k + 2 <= k1; k += 2)
        acc = mfma2(ones, ones, load4(G, Bpad, 16 * c + col, 16 * k + 4 * grp),
                    load4(G, Bpad, 16 * c + col, 16 * (k + 1) + 4 * grp), acc);
      if (k < k1) acc = mfma(ones, load4(G, Bpad, 16 * c + col, 16 * k + 4 * grp), acc);
      const int n = 16 * c + col;
      if (grp == 0 && n < dim) part[off + n] = acc[0];
    }
  }
}

// Gradient of parameter p: the slice partials added in slice order.
__device__ __forceinline__ float grad_sum(const MlpDev& w, int p) {
  float g = 0.f;
#pragma unroll
  for (int s = 0; s < kGradSplit; ++s) g += w.gpart[(size_t)s * kNParams + p];
  return g;
}

__global__ __launch_bounds__(256) void k_mlp_grad_sum(MlpDev w) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < kNParams) w.grad[p] = grad_sum(w, p);
}

// Parameter index -> bf16 copies in both orientations.
__device__ __forceinline__ void write_bf16_copies(const MlpDev& w, int p, float v) {
  const uint16_t h = f2bf(v);
  if (p < kOffB1) {
    const int i = p / kHid, o = p % kHid;
    w.W1t[o * kInPad + i] = h;
  } else if (p < kOffW2) {
    w.b1[p - kOffB1] = v;
  } else if (p < kOffB2) {
    const int q = p - kOffW2, i = q / kHid, o = q % kHid;
    w.W2t[o * kHid + i] = h;
    w.W2n[i * kHid + o] = h;
  } else if (p < kOffW3) {
    w.b2[p - kOffB2] = v;
  } else if (p < kOffB3) {
    const int q = p - kOffW3, i = q / kHid, o = q % kHid;
    w.W3t[o * kHid + i] = h;
    w.W3n[i * kHid + o] = h;
  } else if (p < kOffW4) {
    w.b3[p - kOffB3] = v;
  } else if (p < kOffB4) {
    const int q = p - kOffW4, i = q / kOut, o = q % kOut;
    w.W4t[o * kHid + i] = h;
    w.W4n[i * kOutPad + o] = h;
  } else {
    w.b4[p - kOffB4] = v;
  }
}

// Adam step on the FP32 master weights with the gradient summed from the
// slice partials (update == 0: only refresh the bf16 copies from the
// masters).  c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t).
__global__ __launch_bounds__(256) void k_mlp_adam(MlpDev w, int update, float lr, float b1, float b2, float eps,
                                                  float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kNParams) return;
  float v = w.master[p];
  if (update) {
    const float g = grad_sum(w, p);
    w.grad[p] = g;
    const float m = b1 * w.m1[p] + (1.f - b1) * g;
    const float s = b2 * w.m2[p] + (1.f - b2) * g * g;
    w.m1[p] = m;
    w.m2[p] = s;
    v -= lr * (m * c1) / (sqrtf(s * c2) + eps);
    w.master[p] = v;
  }
  write_bf16_copies(w, p, v);
}

}  // namespace

hipError_t launch_mlp_rows(const MlpDev& w, const float* x, const float* label, const float* log10e, int B, int Bpad,
                           float* out, bool train, hipStream_t st) {
  return launch_mlp_rows_gather(w, x, label, log10e, nullptr, 0, B, Bpad, out, train, st);
}

hipError_t launch_mlp_rows_gather(const MlpDev& w, const float* x, const float* label, const float* log10e,
                                  const int64_t* rows, int64_t n_data, int B, int Bpad, float* out, bool train,
                                  hipStream_t st) {
  const int tiles = Bpad / 16;
  const int grid = (tiles + 3) / 4;
  if (train)
    hipLaunchKernelGGL(k_mlp_rows<true>, dim3(grid), dim3(kRowsNT), 0, st, w, x, label, log10e, rows, n_data, B,
                       Bpad, out);
  else
    hipLaunchKernelGGL(k_mlp_rows<false>, dim3(grid), dim3(kRowsNT), 0, st, w, x, label, log10e, rows, n_data, B,
                       Bpad, out);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpDev& w, int B, int Bpad, float* loss_out, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(kGradBlocks), dim3(64), 0, st, w, B, Bpad, loss_out);
  return hipGetLastError();
}

hipError_t launch_mlp_grad_sum(const MlpDev& w, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_grad_sum, dim3((kNParams + 255) / 256), dim3(256), 0, st, w);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(const MlpDev& w, bool update, float lr, float b1, float b2, float eps, float c1, float c2,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((kNParams + 255) / 256), dim3(256), 0, st, w, update ? 1 : 0, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

}  // namespace rta
