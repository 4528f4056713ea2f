// Internal declarations shared by the kernels and the C-ABI layer of librta.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rta.h"

namespace rta {

constexpr int kMaxPix = RTA_MAX_PIX;
constexpr int kMaxWords = kMaxPix / 64;
constexpr int kNbrCols = 8;  // device neighbour table: int16 [Npad][8], 16 bytes per pixel

// Device-resident tables of one camera type.  Per-pixel arrays are padded
// to Npad entries per gain row so that a lane's pixel group loads as one vector.
struct DevCam {
  int32_t n_pix, n_pix_pad, n_samp, n_gain;
  int32_t window, hg_switch;
  int64_t event_elems;
  float focal;
  int32_t fixed_start;     // first sample of the fixed extraction window
  const int32_t* P256;     // [G][Npad] Q8 pedestal per sample
  const int32_t* thr_pic;  // [G][Npad] Q8 picture threshold (on D)
  const int32_t* thr_bnd;  // [G][Npad] Q8 boundary threshold (on D)
  const float* a;          // [G][Npad] ADC per p.e.
  const float* x;          // [Npad] m
  const float* y;          // [Npad] m
  const int16_t* nbr;      // [Npad][8] neighbour indices, -1 padded
  const uint8_t* border;   // [Npad] 1 if fewer than 6 neighbours
  // The pixels in lattice-row order (rows of equal y, x increasing; any
  // order is correct, this one keeps neighbours of adjacent entries
  // adjacent): lat[p] = the six neighbours' positions in that order, one
  // column per direction (-1 if none), then the pixel index and -1;
  // lpos[j] = the position of pixel j (j itself for padding pixels).
  const int16_t* lat;      // [Npad][8]
  const uint16_t* lpos;    // [Npad]
  // Packet CRC constants of this type (multiplications modulo the CRC
  // polynomial): [0, 256) i*K and [256, 512) i*x^8*K with K = x^(16N), the
  // per-lane finishing factors x^(8 a_l) at [512, 768), then x^(8*body) and
  // 0xFFFF * x^(8*(32+body)) at 768 and 769 (body = 2GTN bytes).
  const uint16_t* crc_tab;
};

constexpr int kCrcTabLen = 770;
constexpr int kDecodeNT = 256;  // lanes per packet; one 16-byte column piece each (rows <= 4096 bytes)
constexpr int kDecodePad = RTA_PACKET_PAD;  // readable bytes required after a packet stream

// Network parameters, packed (matches RTA_MLP_N_PARAMS): W1 [10][64], b1,
// W2 [64][64], b2, W3 [64][64], b3, W4 [64][2], b4, with W[in][out].
constexpr int kNParams = 9154;
constexpr int kGradSplit = 16;  // batch slices of the weight-gradient contraction
constexpr int kOffW1 = 0, kOffB1 = 640, kOffW2 = 704, kOffB2 = 4800, kOffW3 = 4864, kOffB3 = 8960;
constexpr int kOffW4 = 9024, kOffB4 = 9152;

// Device state of the network: FP32 masters and Adam moments, bf16 working
// copies in both orientations (t: [out][in] for the forward A operand, n:
// [in][out] for the backward one), FP32 biases, the feature standardisation,
// and per-batch scratch (feature-major activations / gradients).
struct MlpDev {
  float *master, *m1, *m2, *grad;
  float* gpart;                     // [kGradSplit][kNParams] per-slice partial gradients
  uint16_t *W1t, *W2t, *W3t, *W4t;  // [64][16], [64][64], [64][64], [16][64]
  uint16_t *W2n, *W3n, *W4n;        // [64][64], [64][64], [64][16]
  float *b1, *b2, *b3, *b4;         // [64], [64], [64], [16]
  float *mean, *stdv;               // [16]
  uint16_t *H0, *H1, *H2, *H3, *G1, *G2, *G3, *G4;  // [16|64][Bpad]
  float* loss_row;                  // [Bpad + 1]
};

// Passed by value: the camera tables of all types sit in the kernel argument
// segment and are read with scalar loads at a wave-uniform type index.
struct FusedArgs {
  DevCam cams[RTA_MAX_TYPES];
  int32_t n_types;
  int32_t window;
  int32_t extractor;       // RTA_EXTRACT_*
  int32_t pad_;
  const uint16_t* traces;
  int64_t traces_len;
  const int32_t* tel_type;
  const int64_t* tel_trace_off;
  int64_t n_tel;
  rta_hillas_rec* out;
  unsigned long long* queue;
  uint32_t* status;
  // classification after Hillas (classify != 0): network (have_mlp) and box
  // cuts, per-telescope [score, log10 E] to tel_class
  int32_t classify;
  int32_t have_mlp;
  float* tel_class;
  MlpDev mlp;
  rta_boxcut_desc bc;
};

struct DecodeArgs {
  DevCam cams[RTA_MAX_TYPES];
  int32_t n_types;
  int32_t pad_;
  const uint8_t* bytes;
  int64_t n_bytes;
  const int64_t* pkt_off;
  int32_t* tel_type;
  const int64_t* tel_trace_off;
  int64_t n_pkt;
  uint16_t* pool;
  int64_t pool_elems;
  rta_packet_rec* rec;
  uint32_t* status;
};

// Science alert monitor state on the device.
struct SamDev {
  int32_t grid, n_bins, n_scales, n_offs;
  double t0, bin_s;
  float cell, gamma_cut, sigma_alert, r_on2;
  int32_t scales[RTA_SAM_MAX_SCALES];
  int32_t* counts;      // [n_bins][grid][grid]
  int32_t* win;         // [n_scales][grid][grid] window sums
  const int32_t* offs;  // [n_offs] disc / ring offsets: (dx + 128) | (dy + 128) << 8 | kind << 16 (1 on, 2 off)
};

struct EventArgs {
  rta_boxcut_desc bc;
  MlpDev mlp;
  int32_t have_mlp;   // network attached (else box cuts only, when have_box)
  int32_t have_box;   // classification enabled
  float focal[RTA_MAX_TYPES];
  int32_t n_types;
  float max_width_ratio;
  float max_cond;
  int32_t pad_;
  const int64_t* evt_tel_off;
  const int32_t* tel_type;
  int64_t n_evt;
  int64_t n_tel;
  rta_hillas_rec* tel;
  rta_event_rec* out;
  const float* tel_class; // [n_tel][2] or null: telescopes already classified
  uint64_t* done_clock;   // [n_evt] or null: device clock at each record write
  uint32_t* status;
};

hipError_t launch_mlp_rows(const MlpDev& w, const float* x, const float* label, const float* log10e, int B, int Bpad,
                           float* out, bool train, hipStream_t st);
hipError_t launch_mlp_grad(const MlpDev& w, int B, int Bpad, float* loss_out, hipStream_t st);
hipError_t launch_mlp_grad_sum(const MlpDev& w, hipStream_t st);
hipError_t launch_mlp_adam(const MlpDev& w, bool update, float lr, float b1, float b2, float eps, float c1, float c2,
                           hipStream_t st);

// Kernel launchers (reco.hip).  Each returns the launch status.
hipError_t launch_calibrate(const DevCam& c, int extractor, const uint16_t* traces, int64_t n_evt, int32_t* S,
                            int32_t* D, uint8_t* sstar, uint8_t* peak, uint8_t* gain, float* q, float* t,
                            hipStream_t st);
// levels: NULL for the camera's threshold tables, else the two levels whose
// thresholds the kernel forms per pixel as the camera creation does.
hipError_t launch_clean(const DevCam& c, const rta_clean_params* levels, const int32_t* D, const uint8_t* gain,
                        int64_t n_evt, uint8_t* mask, hipStream_t st);
// Charges from q (p.e.) or, when q is NULL, from D (Q8) and gain.
hipError_t launch_hillas(const DevCam& c, const float* q, const int32_t* D, const float* t, const uint8_t* mask,
                         const uint8_t* gain, int64_t n_evt, rta_hillas_rec* out, hipStream_t st);
hipError_t launch_decode(const DecodeArgs& a, hipStream_t st);
// Health accumulation: at most kHealthParts workgroups, each leaving its
// per-pixel sums in a partial block [3][G][Npad] of the camera's scratch.
constexpr int kHealthParts = 512;
hipError_t launch_health(const DevCam& c, const uint16_t* traces, int64_t n_evt, const rta_health_params& p,
                         uint64_t* part, uint64_t* acc, rta_pixel_health* pix, rta_camera_health* out,
                         hipStream_t st);
hipError_t launch_sam_clear(const SamDev& d, hipStream_t st);
hipError_t launch_sam_fill(const SamDev& d, const rta_event_rec* evt, const double* t, int64_t n, hipStream_t st);
hipError_t launch_sam_search(const SamDev& d, int end_bin, double* sig, int32_t* n_on, int32_t* n_off,
                             rta_sam_alert* alerts, int max_alerts, int32_t* n_alerts, hipStream_t st);
hipError_t launch_queue_reset(unsigned long long* queue, hipStream_t st);
hipError_t launch_fused(const FusedArgs& a, const rta_schedule& s, int n_cu, hipStream_t st);
hipError_t launch_event(const EventArgs& a, hipStream_t st);
hipError_t launch_stamp(uint64_t* slot, hipStream_t st);
hipError_t launch_features(const rta_hillas_rec* rec, int64_t n, float* x, hipStream_t st);
hipError_t launch_classify(const MlpDev& w, bool have_mlp, const rta_boxcut_desc& bc, const rta_hillas_rec* rec,
                           int64_t n, float* out, hipStream_t st);

bool window_supported(int w);
bool extractor_supported(int ex);
bool schedule_supported(const rta_schedule& s);
int list_schedules(rta_schedule* out, int cap);

}  // namespace rta
