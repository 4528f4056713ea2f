// HIP decode of the DL0 telemetry packet stream for gfx950 (CDNA4).
//
// The real-time analysis receives camera events as a byte stream formatted
// like space telemetry source packets (paper, Section 5); the packet layout
// is defined in rta.h.  One workgroup decodes one packet: the header is read
// by every lane (uniform), then lane l owns bytes [16 l, 16 l + 16) of every
// sample row (G*T rows of 2N bytes, N <= 2048 so a row has at most 256
// pieces).  Per row the lane
//   * loads its 16 bytes (two aligned loads and a funnel shift: packets are
//     only 2-byte aligned in the stream),
//   * swaps the big-endian samples to little-endian and stores them as one
//     16-byte write into the [G][T][Npad] pool slot (zero pad columns),
//   * folds the bytes into its CRC share.
// CRC over GF(2): the register after a message M from register 0 is
// crc0(M) = M(x) x^16 mod P, and crc0(A || B) = crc0(A) x^(8|B|) + crc0(B).
// The lane's pieces recur every 2N bytes, so its share is the Horner sum
// h <- h*K + crc0(piece) with K = x^(16N) (a table product), times x^(8 a_l)
// for the a_l bytes after its piece in the last row.  The shares, the
// header's crc0 times x^(8*body) and the initial register's 0xFFFF *
// x^(8*(32+body)) XOR to the packet's CRC.
#include "rta_internal.h"

namespace rta {
namespace {

constexpr int kWave = 64;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Product modulo the CRC polynomial (bit-serial, used once per lane).
__device__ __forceinline__ uint32_t gf_mul_dev(uint32_t a, uint32_t b) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 15; i >= 0; --i) {
    r <<= 1;
    if (r & 0x10000u) r ^= 0x11021u;
    if ((b >> i) & 1u) r ^= a;
  }
  return r;
}

// XOR over the wavefront, valid in lane 63 (DPP lane moves only).
__device__ __forceinline__ uint32_t wave_xor_last(uint32_t v) {
  v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
  v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

// Sixteen stream bytes from byte offset off (2-byte aligned) of the buffer:
// two aligned loads and a funnel shift by 0 or 2 bytes.
__device__ __forceinline__ void load16(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t (&w)[4]) {
  const uint32_t a = off & ~3u, sh = (off & 3u) * 8u;
  const u32x4 d = __builtin_amdgcn_raw_buffer_load_b128(r, (int)a, 0, 0);
  const uint32_t e = __builtin_amdgcn_raw_buffer_load_b32(r, (int)(a + 16u), 0, 0);
  w[0] = __builtin_amdgcn_alignbit(d[1], d[0], sh);
  w[1] = __builtin_amdgcn_alignbit(d[2], d[1], sh);
  w[2] = __builtin_amdgcn_alignbit(d[3], d[2], sh);
  w[3] = __builtin_amdgcn_alignbit(e, d[3], sh);
}

__device__ __forceinline__ uint32_t byte_of(const uint32_t (&w)[8], int i) { return (w[i >> 2] >> ((i & 3) * 8)) & 0xFFu; }

__global__ __launch_bounds__(kDecodeNT) void k_decode_packets(DecodeArgs a) {
  __shared__ uint16_t T0[256], T1[256], KL[256], KH[256];
  __shared__ uint32_t share[kDecodeNT / kWave];
  const int lane = threadIdx.x;
  const int64_t p = blockIdx.x;
  // CRC byte tables from the polynomial: T0[i] = i x^16 mod P, T1[i] = i x^24 mod P
  {
    uint32_t r = (uint32_t)lane << 8;
#pragma unroll
    for (int b = 0; b < 8; ++b) r = (r & 0x8000u) ? ((r << 1) ^ 0x1021u) & 0xFFFFu : (r << 1) & 0xFFFFu;
    T0[lane] = (uint16_t)r;
  }
  __syncthreads();
  {
    const uint32_t v = T0[lane];
    T1[lane] = (uint16_t)(((v << 8) ^ T0[v >> 8]) & 0xFFFFu);
  }
  // header: 32 bytes at po (every lane, uniform)
  const int64_t po = uniform64(a.pkt_off[p]);
  // an offset that leaves no room for a header inside the stream reads
  // nothing (an empty buffer range: every load returns zero) and is flagged
  const bool po_ok = po >= 0 && po + 34 <= a.n_bytes;
  const int64_t base = po_ok ? (po & ~int64_t(15)) : 0;
  // every load stays below n_bytes + 32 (the caller keeps those 32 bytes
  // readable): loads are 16-byte pieces at 4-byte aligned addresses, so the
  // pieces at the end of a packet reach past it into the next packet or the
  // padding, and a piece straddling the buffer's range would read as zero
  const int64_t avail = po_ok ? a.n_bytes + kDecodePad - base : 0;
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t*>(a.bytes + base), 0, (int)(avail > 0x7ffffff0LL ? 0x7ffffff0LL : (avail > 0 ? avail : 0)),
      0x00020000);
  const uint32_t o0 = po_ok ? (uint32_t)(po - base) : 0u;
  uint32_t hw[8];
  {
    uint32_t t[4];
    load16(r, o0, t);
    hw[0] = t[0]; hw[1] = t[1]; hw[2] = t[2]; hw[3] = t[3];
    load16(r, o0 + 16u, t);
    hw[4] = t[0]; hw[5] = t[1]; hw[6] = t[2]; hw[7] = t[3];
  }
  auto g8 = [&](int i) { return byte_of(hw, i); };
  auto g16 = [&](int i) { return (g8(i) << 8) | g8(i + 1); };
  auto g32 = [&](int i) { return (g16(i) << 16) | g16(i + 2); };
  // header values are the same in every lane; make that explicit (scalar
  // registers: kernel-argument table indexing and loop bounds stay scalar)
  const uint32_t pid = __builtin_amdgcn_readfirstlane(g16(0)), seq = __builtin_amdgcn_readfirstlane(g16(2));
  const uint32_t dlen = __builtin_amdgcn_readfirstlane(g32(4));
  const uint32_t ty = __builtin_amdgcn_readfirstlane(g8(11)), N = __builtin_amdgcn_readfirstlane(g16(18));
  const uint32_t T = __builtin_amdgcn_readfirstlane(g16(20)), G = __builtin_amdgcn_readfirstlane(g8(22));
  uint32_t flags = po_ok ? 0u : RTA_PKT_HEADER_BAD;
  const uint64_t body = 2ull * N * T * G;
  if ((pid >> 11) != 1u || (seq >> 14) != 3u || g8(8) != 0x10u || g8(9) != 210u || g8(10) != 1u || g8(23) != 0u ||
      (uint64_t)dlen + 9ull != 34ull + body || po + 34 + (int64_t)body > a.n_bytes)
    flags |= RTA_PKT_HEADER_BAD;
  const int tt = __builtin_amdgcn_readfirstlane(a.tel_type[p]);
  const int64_t slot = uniform64(a.tel_trace_off[p]);
  if ((int)ty >= a.n_types || tt != (int)ty) {
    flags |= RTA_PKT_TYPE_BAD;
  } else {
    const DevCam& c = a.cams[ty];
    if ((uint32_t)c.n_pix != N || (uint32_t)c.n_samp != T || (uint32_t)c.n_gain != G || slot < 0 || (slot & 7) ||
        slot + c.event_elems > a.pool_elems)
      flags |= RTA_PKT_TYPE_BAD;
  }
  flags = __builtin_amdgcn_readfirstlane(flags);
  uint32_t crc_calc = 0, crc_stored = 0;
  if (flags == 0) {
    const DevCam& c = a.cams[ty];
    KL[lane] = c.crc_tab[lane];
    KH[lane] = c.crc_tab[256 + lane];
    __syncthreads();
    const uint32_t row = 2u * N, rows = T * G, np = (uint32_t)c.n_pix_pad;
    const uint32_t lo = 16u * (uint32_t)lane;
    const bool act = lo < row;
    const int nb = act ? (int)min(16u, row - lo) : 0;  // bytes of this lane's piece (even)
    uint16_t* dst = a.pool + slot + 8 * lane;
    uint32_t h = 0;
    uint32_t in = o0 + 32u + lo;
    // four rows in flight per lane: loads past the packet's last row read the
    // next packet or the padding and are ignored
    constexpr int R = 4;
    for (uint32_t k0 = 0; k0 < rows; k0 += R, in += R * row) {
      uint32_t w[R][4];
#pragma unroll
      for (int j = 0; j < R; ++j) load16(r, in + (uint32_t)j * row, w[j]);
      // CRC shares of the R pieces, two bytes (one sample) per step, the R
      // independent lookup chains interleaved; whole pieces take the
      // branch-free path, only the last lane of a row can hold fewer bytes
      uint32_t cc[R];
#pragma unroll
      for (int j = 0; j < R; ++j) cc[j] = 0;
      if (nb == 16) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
#pragma unroll
          for (int j = 0; j < R; ++j) {
            const uint32_t b0 = (w[j][i >> 1] >> ((i & 1) * 16)) & 0xFFu;
            const uint32_t b1 = (w[j][i >> 1] >> ((i & 1) * 16 + 8)) & 0xFFu;
            cc[j] = (uint32_t)T1[(cc[j] >> 8) ^ b0] ^ (uint32_t)T0[(cc[j] & 0xFFu) ^ b1];
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          if (2 * i < nb) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
              const uint32_t b0 = (w[j][i >> 1] >> ((i & 1) * 16)) & 0xFFu;
              const uint32_t b1 = (w[j][i >> 1] >> ((i & 1) * 16 + 8)) & 0xFFu;
              cc[j] = (uint32_t)T1[(cc[j] >> 8) ^ b0] ^ (uint32_t)T0[(cc[j] & 0xFFu) ^ b1];
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (k0 + j >= rows) continue;
        h = (uint32_t)KH[h >> 8] ^ (uint32_t)KL[h & 0xFFu] ^ cc[j];
        // big-endian samples -> little-endian, zero beyond the row
        u32x4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t s = __builtin_amdgcn_perm(w[j][q], w[j][q], 0x02030001u);
          v[q] = 4 * q < nb ? (4 * q + 2 < nb ? s : (s & 0xFFFFu)) : 0u;
        }
        if (act) *reinterpret_cast<u32x4*>(dst + (size_t)(k0 + j) * np) = v;
      }
    }
    uint32_t share_l = act ? gf_mul_dev(h, c.crc_tab[512 + lane]) : 0u;
    share_l = wave_xor_last(share_l);
    if ((lane & (kWave - 1)) == kWave - 1) share[lane / kWave] = share_l;
    __syncthreads();
    if (lane == 0) {
      uint32_t hc = 0;
#pragma unroll
      for (int i = 0; i < 32; i += 2) hc = (uint32_t)T1[(hc >> 8) ^ g8(i)] ^ (uint32_t)T0[(hc & 0xFFu) ^ g8(i + 1)];
      crc_calc = gf_mul_dev(hc, c.crc_tab[768]) ^ c.crc_tab[769];
#pragma unroll
      for (int w = 0; w < kDecodeNT / kWave; ++w) crc_calc ^= share[w];
      uint32_t t2[4];
      load16(r, o0 + 32u + (uint32_t)body, t2);
      crc_stored = ((t2[0] & 0xFFu) << 8) | ((t2[0] >> 8) & 0xFFu);
      if (crc_calc != crc_stored) flags |= RTA_PKT_CRC_BAD;
    }
  }
  if (lane == 0) {
    if (flags) {
      a.tel_type[p] = -1;
      atomicOr(a.status, RTA_STATUS_BAD_PACKET);
    }
    if (a.rec) {
      rta_packet_rec rc;
      rc.event_number = ((uint64_t)g32(24) << 32) | g32(28);
      rc.coarse_time = g32(12);
      rc.fine_time = (uint16_t)g16(16);
      rc.apid = (uint16_t)(pid & 0x7FFu);
      rc.seq_count = (uint16_t)(seq & 0x3FFFu);
      rc.cam_type = (uint16_t)ty;
      rc.flags = flags;
      rc.crc_stored = (uint16_t)crc_stored;
      rc.crc_computed = (uint16_t)crc_calc;
      rc.pad_ = 0;
      a.rec[p] = rc;
    }
  }
}

}  // namespace

hipError_t launch_decode(const DecodeArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_decode_packets, dim3((unsigned)a.n_pkt), dim3(kDecodeNT), 0, st, a);
  return hipGetLastError();
}

}  // namespace rta
