// C ABI of librta: argument validation, camera tables, pipelines, graphs.
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lattice.h"
#include "mlp_launch.h"
#include "rta_internal.h"

struct rta_camera {
  rta::DevCam dev;
  void* dmem = nullptr;
  rta_camera_info info{};
  int device = 0;
  uint64_t* health_acc = nullptr;   // [3][G][Npad] health totals (s1, s2, n_sat), inside dmem
  uint64_t* health_part = nullptr;  // [kHealthParts][3][G][Npad] per-workgroup partial sums, inside dmem
  double max_a = 0.0;                // largest adc_per_pe of the camera (threshold range checks)
};

struct rta_pipeline {
  std::vector<rta_camera*> cams;
  rta_mlp* mlp = nullptr;        // attached network (not owned)
  bool have_box = false;
  rta_boxcut_desc bc{};
  rta_pipeline_params params{};
  rta_schedule sched{};
  int window = 0;
  int n_cu = 0;
  int device = 0;
  unsigned long long* d_queue = nullptr;  // work-queue counter
  uint32_t* d_status = nullptr;           // RTA_STATUS_* bits
  hipStream_t capture_stream = nullptr;
  std::string tune_key;                   // "<arch>|e<extractor>w<window>|<N>x<T>x<G>;..."
  std::string tune_cache;                 // tune cache path ("" without one)
  bool untuned = false;                   // a cache was given but held no schedule yet
};

struct rta_sam {
  rta::SamDev dev{};
  void* dmem = nullptr;
  int device = 0;
};

struct rta_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct rta_mlp {
  rta::MlpDev dev{};
  void* dmem = nullptr;
  int max_batch = 0, bpad_max = 0;
  int64_t last_B = 0;  // batch of the last loss_grad / train_step pass (0: none yet)
  float lr = 1e-3f, beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  int64_t step = 0;
  bool has_params = false;
};

namespace {

thread_local std::string g_err;

rta_status fail(rta_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define RTA_HIP(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(RTA_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

size_t round256(size_t v) { return (v + 255) & ~size_t(255); }

// Product of two residues modulo the packet CRC polynomial x^16+x^12+x^5+1
// (polynomials over GF(2), bit i = coefficient of x^i).
uint32_t gf_mul(uint32_t a, uint32_t b) {
  uint32_t r = 0;
  for (int i = 15; i >= 0; --i) {
    r <<= 1;
    if (r & 0x10000u) r ^= 0x11021u;
    if ((b >> i) & 1u) r ^= a;
  }
  return r;
}

// x^(8n) modulo the CRC polynomial.
uint32_t gf_pow8(uint64_t n) {
  uint32_t res = 1, base = 0x100;
  while (n) {
    if (n & 1) res = gf_mul(res, base);
    base = gf_mul(base, base);
    n >>= 1;
  }
  return res;
}

// Constants of the parallel packet CRC for one camera type (layout in DevCam).
void crc_tables(int N, int T, int G, uint16_t* t) {
  const uint64_t row = 2ull * (uint64_t)N, body = row * (uint64_t)T * (uint64_t)G;
  const uint32_t K = gf_pow8(row);
  for (uint32_t i = 0; i < 256; ++i) {
    t[i] = (uint16_t)gf_mul(i, K);
    t[256 + i] = (uint16_t)gf_mul(i << 8, K);
  }
  for (int l = 0; l < rta::kDecodeNT; ++l) {
    const uint64_t lo = 16ull * (uint64_t)l;
    t[512 + l] = (uint16_t)(lo < row ? gf_pow8(row - std::min<uint64_t>(lo + 16, row)) : 1u);
  }
  t[768] = (uint16_t)gf_pow8(body);
  t[769] = (uint16_t)gf_mul(0xFFFFu, gf_pow8(32 + body));
}

void fill_event_args(const rta_pipeline* pipe, rta::EventArgs& ea);


// Scratch of rta_process_batch_noalloc: the work-queue counter at byte
// kScratchQueue and the status word at byte kScratchStatus.  One copy per GPU
// (the runtime places a device variable on every device that loads the
// library), held until the process ends.  Host code never uses the name
// `scratch` as an address: noalloc_scratch() resolves each device's copy once.
constexpr size_t kScratchQueue = 0, kScratchStatus = 64;
static_assert(kScratchStatus + sizeof(uint32_t) <= RTA_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds its size");
static __device__ __align__(256) uint8_t scratch[RTA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on device dev (which must be current): looked
// up by hipGetSymbolAddress on the first call for that device, then cached.
rta_status noalloc_scratch(int dev, uint8_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(RTA_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(RTA_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<uint8_t*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return RTA_OK;
}

// Clears the counter and the status word of a scratch copy (a kernel, not a
// memset, so that the call can be captured into a graph).
__global__ void k_scratch_reset(unsigned long long* queue, uint32_t* status) {
  if (threadIdx.x == 0) {
    *queue = 0ull;
    *status = 0u;
  }
}

__global__ void k_status_copy(const uint32_t* status, uint32_t* out) {
  if (threadIdx.x == 0) *out = *status;
}

// Launches of one batch; queue: the work-queue counter, status: the status
// word the kernels OR their RTA_STATUS_* bits into.
rta_status launch_batch(const rta_pipeline* pipe, const rta_batch* b, rta_hillas_rec* tel_out,
                        rta_event_rec* evt_out, unsigned long long* queue, uint32_t* status, hipStream_t st) {
  rta::FusedArgs fa;
  std::memset(&fa, 0, sizeof(fa));
  for (size_t i = 0; i < pipe->cams.size(); ++i) fa.cams[i] = pipe->cams[i]->dev;
  fa.n_types = (int32_t)pipe->cams.size();
  fa.window = pipe->window;
  fa.extractor = pipe->params.extractor;
  fa.pad_ = 0;
  fa.traces = b->traces;
  fa.traces_len = b->traces_len;
  fa.tel_type = b->tel_type;
  fa.tel_trace_off = b->tel_trace_off;
  fa.n_tel = b->n_tel;
  fa.out = tel_out;
  fa.queue = queue;
  fa.status = status;
  if (b->tel_class && pipe->have_box) {
    fa.classify = 1;
    fa.tel_class = b->tel_class;
    fa.bc = pipe->bc;
    fa.have_mlp = pipe->mlp ? 1 : 0;
    if (pipe->mlp) fa.mlp = pipe->mlp->dev;
  }
  if (b->n_tel > 0) {
    RTA_HIP(rta::launch_queue_reset(queue, st));
    RTA_HIP(rta::launch_fused(fa, pipe->sched, pipe->n_cu, st));
  }
  if (pipe->params.do_stereo && b->n_evt > 0) {
    rta::EventArgs ea;
    fill_event_args(pipe, ea);
    ea.evt_tel_off = b->evt_tel_off;
    ea.tel_type = b->tel_type;
    ea.n_evt = b->n_evt;
    ea.n_tel = b->n_tel;
    ea.tel = tel_out;
    ea.out = evt_out;
    ea.tel_class = fa.classify ? b->tel_class : nullptr;
    ea.done_clock = b->evt_done_clock;
    ea.status = status;
    RTA_HIP(rta::launch_event(ea, st));
  }
  return RTA_OK;
}

// ---- schedule tune cache (text file, one "<key>\t<4 ints>\t<ms>" line per key)

std::mutex g_tune_file_mu;  // serialises read-modify-write of cache files within the process

bool parse_tune_line(const std::string& line, std::string* key, rta_schedule* s, float* ms) {
  if (line.empty() || line[0] == '#') return false;
  const size_t tab = line.find('\t');
  if (tab == std::string::npos || tab == 0) return false;
  rta_schedule v{};
  float t = 0.f;
  char extra = 0;
  if (std::sscanf(line.c_str() + tab + 1, " %d %d %d %d %f %c", &v.pix_per_lane, &v.waves_per_wg, &v.wg_per_cu,
                  &v.chunk, &t, &extra) != 5)
    return false;
  *key = line.substr(0, tab);
  *s = v;
  *ms = t;
  return true;
}

// Lines of a text file without their line breaks; false if it cannot be opened.
bool read_lines(const char* path, std::vector<std::string>* lines) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  std::string cur;
  char buf[1024];
  while (std::fgets(buf, sizeof(buf), f)) {
    cur += buf;
    if (!cur.empty() && cur.back() == '\n') {
      cur.pop_back();
      if (!cur.empty() && cur.back() == '\r') cur.pop_back();
      lines->push_back(cur);
      cur.clear();
    }
  }
  if (!cur.empty()) lines->push_back(cur);
  std::fclose(f);
  return true;
}

rta_status make_tune_key(const rta_pipeline* p, std::string* key) {
  hipDeviceProp_t prop;
  RTA_HIP(hipGetDeviceProperties(&prop, p->device));
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  char buf[64];
  std::snprintf(buf, sizeof(buf), "|e%dw%d|", (int)p->params.extractor, p->window);
  std::string k = arch + buf;
  for (size_t i = 0; i < p->cams.size(); ++i) {
    const rta_camera_info& c = p->cams[i]->info;
    std::snprintf(buf, sizeof(buf), "%s%dx%dx%d", i ? ";" : "", (int)c.n_pix, (int)c.n_samp, (int)c.n_gain);
    k += buf;
  }
  *key = k;
  return RTA_OK;
}

rta_status check_batch(const rta_pipeline* pipe, const rta_batch* b, const rta_hillas_rec* tel_out,
                       const rta_event_rec* evt_out, bool need_schedule = true) {
  if (!pipe || !b) return fail(RTA_E_INVALID_ARG, "null pipeline or batch");
  if (need_schedule && pipe->untuned)
    return fail(RTA_E_UNTUNED, "the tune cache holds no schedule for " + pipe->tune_key +
                                   "; run rta_pipeline_tune or set a schedule");
  if (b->n_tel < 0 || b->n_evt < 0 || b->traces_len < 0) return fail(RTA_E_INVALID_ARG, "negative batch size");
  if (b->n_tel > 0) {
    if (!b->traces || !b->tel_type || !b->tel_trace_off || !tel_out)
      return fail(RTA_E_INVALID_ARG, "null trace pool, descriptor or output pointer");
    if (!aligned16(b->traces)) return fail(RTA_E_INVALID_ARG, "trace pool must be 16-byte aligned");
  }
  if (b->tel_class && !pipe->have_box)
    return fail(RTA_E_INVALID_ARG, "tel_class needs a classifier attached to the pipeline");
  if (pipe->params.do_stereo && b->n_evt > 0) {
    if (!b->evt_tel_off || !evt_out || !tel_out) return fail(RTA_E_INVALID_ARG, "null event offsets or output");
    if ((int64_t)(b->n_evt + 3) / 4 > 0x7fffffffLL) return fail(RTA_E_SHAPE, "too many events for one launch");
  }
  return RTA_OK;
}

}  // namespace

extern "C" {

const char* rta_status_str(rta_status s) {
  switch (s) {
    case RTA_OK: return "ok";
    case RTA_E_INVALID_ARG: return "invalid argument";
    case RTA_E_SHAPE: return "unsupported shape";
    case RTA_E_HIP: return "HIP runtime error";
    case RTA_E_NOMEM: return "out of memory";
    case RTA_E_UNSUPPORTED: return "unsupported option";
    case RTA_E_UNTUNED: return "no tuned schedule";
  }
  return "unknown status";
}

const char* rta_last_error(void) { return g_err.c_str(); }

int32_t rta_version(void) { return RTA_VERSION; }

rta_status rta_device_clock_hz(int64_t* hz) {
  if (!hz) return fail(RTA_E_INVALID_ARG, "null hz");
  int dev = 0, khz = 0;
  RTA_HIP(hipGetDevice(&dev));
  RTA_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) return fail(RTA_E_HIP, "device reports no clock rate");
  *hz = (int64_t)khz * 1000;
  return RTA_OK;
}

rta_status rta_device_stamp(uint64_t* slot, rta_stream stream) {
  if (!slot) return fail(RTA_E_INVALID_ARG, "null slot");
  RTA_HIP(rta::launch_stamp(slot, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_device_cus(int32_t* n_cu) {
  if (!n_cu) return fail(RTA_E_INVALID_ARG, "null n_cu");
  int dev = 0, v = 0;
  RTA_HIP(hipGetDevice(&dev));
  RTA_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev));
  *n_cu = v;
  return RTA_OK;
}

rta_status rta_camera_create(const rta_camera_desc* d, rta_camera** out) {
  if (!d || !out) return fail(RTA_E_INVALID_ARG, "null descriptor or output handle");
  *out = nullptr;
  const int N = d->n_pix, T = d->n_samp, G = d->n_gain, w = d->window, M = d->max_nbr;
  if (N < 1 || N > RTA_MAX_PIX) return fail(RTA_E_SHAPE, "n_pix must be in [1, RTA_MAX_PIX]");
  if (G != 1 && G != 2) return fail(RTA_E_SHAPE, "n_gain must be 1 or 2");
  if (!rta::window_supported(w)) return fail(RTA_E_SHAPE, "window not in the compiled set");
  if (T < w || T > RTA_MAX_SAMP) return fail(RTA_E_SHAPE, "n_samp must be in [window, RTA_MAX_SAMP]");
  if (M < 0 || M > 6) return fail(RTA_E_SHAPE, "max_nbr must be in [0, 6]");
  if (!d->pix_x || !d->pix_y || !d->ped || !d->adc_per_pe || (M > 0 && !d->nbr))
    return fail(RTA_E_INVALID_ARG, "null table pointer");
  if (!std::isfinite(d->t_pic) || !std::isfinite(d->t_bnd) || d->t_bnd > d->t_pic)
    return fail(RTA_E_INVALID_ARG, "cleaning levels must be finite with t_bnd <= t_pic");
  if (!std::isfinite(d->focal_m) || !(d->focal_m > 0.f)) return fail(RTA_E_INVALID_ARG, "focal length must be > 0");
  if (d->fixed_start < 0 || d->fixed_start > T - w)
    return fail(RTA_E_SHAPE, "fixed_start must be in [0, n_samp - window]");
  const int Np = (N + 7) & ~7;
  std::vector<int32_t> P(G * Np, 0), Tp(G * Np, 0x7fffffff), Tb(G * Np, 0x7fffffff);
  double max_a = 0.0;
  std::vector<float> A(G * Np, 1.f), X(Np, 0.f), Y(Np, 0.f);
  std::vector<int16_t> nb(Np * rta::kNbrCols, -1);
  std::vector<uint8_t> border(Np, 0);
  std::vector<uint16_t> crc(rta::kCrcTabLen, 0);
  crc_tables(N, T, G, crc.data());
  for (int g = 0; g < G; ++g)
    for (int i = 0; i < N; ++i) {
      const float ped = d->ped[g * N + i], a = d->adc_per_pe[g * N + i];
      if (!std::isfinite(ped) || std::fabs(ped) > 65536.f) return fail(RTA_E_INVALID_ARG, "pedestal out of range");
      if (!std::isfinite(a) || !(a > 0.f)) return fail(RTA_E_INVALID_ARG, "adc_per_pe must be > 0");
      // Q8 pedestal, nearest with ties to even (256 * ped is exact in double).
      P[g * Np + i] = (int32_t)std::nearbyint(256.0 * (double)ped);
      // 256 * a * level: a product of two floats is exact in double, so the
      // ceiling is the exact integer threshold on D.
      const double tp = std::ceil(256.0 * (double)a * (double)d->t_pic);
      const double tb = std::ceil(256.0 * (double)a * (double)d->t_bnd);
      if (std::fabs(tp) > 2.0e9 || std::fabs(tb) > 2.0e9) return fail(RTA_E_INVALID_ARG, "threshold overflow");
      Tp[g * Np + i] = (int32_t)tp;
      Tb[g * Np + i] = (int32_t)tb;
      A[g * Np + i] = a;
      max_a = std::max(max_a, (double)a);
    }
  for (int i = 0; i < N; ++i) {
    X[i] = d->pix_x[i];
    Y[i] = d->pix_y[i];
    int cnt = 0;
    for (int k = 0; k < M; ++k) {
      const int j = d->nbr[(size_t)i * M + k];
      if (j < -1 || j >= N || j == i) return fail(RTA_E_INVALID_ARG, "neighbour index out of range");
      if (j >= 0) nb[(size_t)i * rta::kNbrCols + cnt++] = (int16_t)j;
    }
    border[i] = cnt < 6 ? 1 : 0;
  }
  static_assert(rta::kLatCols == rta::kNbrCols, "lattice rows share the neighbour table's width");
  std::vector<int16_t> lat(Np * rta::kNbrCols, -1);
  std::vector<uint16_t> lpos(Np, 0);
  rta::lattice_order(N, Np, X.data(), Y.data(), nb.data(), lat.data(), lpos.data());
  // one device allocation, 256-byte aligned sub-arrays
  const size_t oP = 0, oTp = oP + round256(P.size() * 4), oTb = oTp + round256(Tp.size() * 4);
  const size_t oA = oTb + round256(Tb.size() * 4), oX = oA + round256(A.size() * 4);
  const size_t oY = oX + round256(X.size() * 4), oN = oY + round256(Y.size() * 4);
  const size_t oB = oN + round256(nb.size() * 2), oC = oB + round256(border.size());
  const size_t oL = oC + round256(crc.size() * 2), oLP = oL + round256(lat.size() * 2);
  const size_t oH = oLP + round256(lpos.size() * 2);
  const size_t oHP = oH + round256((size_t)3 * G * Np * 8);
  const size_t total = oHP + round256((size_t)rta::kHealthParts * 3 * G * Np * 8);
  // tables are copied from the host; the health scratch after them is
  // written by the health kernels before it is read
  std::vector<uint8_t> host(oH, 0);
  std::memcpy(host.data() + oP, P.data(), P.size() * 4);
  std::memcpy(host.data() + oTp, Tp.data(), Tp.size() * 4);
  std::memcpy(host.data() + oTb, Tb.data(), Tb.size() * 4);
  std::memcpy(host.data() + oA, A.data(), A.size() * 4);
  std::memcpy(host.data() + oX, X.data(), X.size() * 4);
  std::memcpy(host.data() + oY, Y.data(), Y.size() * 4);
  std::memcpy(host.data() + oN, nb.data(), nb.size() * 2);
  std::memcpy(host.data() + oB, border.data(), border.size());
  std::memcpy(host.data() + oC, crc.data(), crc.size() * 2);
  std::memcpy(host.data() + oL, lat.data(), lat.size() * 2);
  std::memcpy(host.data() + oLP, lpos.data(), lpos.size() * 2);
  rta_camera* cam = new (std::nothrow) rta_camera();
  if (!cam) return fail(RTA_E_NOMEM, "host allocation failed");
  if (hipGetDevice(&cam->device) != hipSuccess || hipMalloc(&cam->dmem, total) != hipSuccess) {
    delete cam;
    return fail(RTA_E_NOMEM, "device allocation for camera tables failed");
  }
  if (hipMemcpy(cam->dmem, host.data(), oH, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(cam->dmem);
    delete cam;
    return fail(RTA_E_HIP, "copy of camera tables failed");
  }
  uint8_t* base = static_cast<uint8_t*>(cam->dmem);
  rta::DevCam& c = cam->dev;
  c.n_pix = N;
  c.n_pix_pad = Np;
  c.n_samp = T;
  c.n_gain = G;
  c.window = w;
  c.hg_switch = d->hg_switch_adc;
  c.event_elems = (int64_t)G * T * Np;
  c.focal = d->focal_m;
  c.fixed_start = d->fixed_start;
  c.P256 = reinterpret_cast<const int32_t*>(base + oP);
  c.thr_pic = reinterpret_cast<const int32_t*>(base + oTp);
  c.thr_bnd = reinterpret_cast<const int32_t*>(base + oTb);
  c.a = reinterpret_cast<const float*>(base + oA);
  c.x = reinterpret_cast<const float*>(base + oX);
  c.y = reinterpret_cast<const float*>(base + oY);
  c.nbr = reinterpret_cast<const int16_t*>(base + oN);
  c.border = base + oB;
  c.crc_tab = reinterpret_cast<const uint16_t*>(base + oC);
  c.lat = reinterpret_cast<const int16_t*>(base + oL);
  c.lpos = reinterpret_cast<const uint16_t*>(base + oLP);
  cam->health_acc = reinterpret_cast<uint64_t*>(base + oH);
  cam->health_part = reinterpret_cast<uint64_t*>(base + oHP);
  cam->info = rta_camera_info{N, Np, T, G, w, d->fixed_start, c.event_elems};
  cam->max_a = max_a;
  *out = cam;
  return RTA_OK;
}

rta_status rta_camera_destroy(rta_camera* cam) {
  if (!cam) return RTA_OK;
  if (cam->dmem) (void)hipFree(cam->dmem);
  delete cam;
  return RTA_OK;
}

rta_status rta_camera_get_info(const rta_camera* cam, rta_camera_info* info) {
  if (!cam || !info) return fail(RTA_E_INVALID_ARG, "null camera or info");
  *info = cam->info;
  return RTA_OK;
}

rta_status rta_calibrate(const rta_camera* cam, const uint16_t* traces, int64_t n_evt, int32_t* S, int32_t* D,
                         uint8_t* sstar, uint8_t* peak, uint8_t* gain, float* q, float* t, rta_stream stream) {
  return rta_calibrate_ex(cam, RTA_EXTRACT_SLIDING, traces, n_evt, S, D, sstar, peak, gain, q, t, stream);
}

rta_status rta_calibrate_ex(const rta_camera* cam, int32_t extractor, const uint16_t* traces, int64_t n_evt,
                            int32_t* S, int32_t* D, uint8_t* sstar, uint8_t* peak, uint8_t* gain, float* q,
                            float* t, rta_stream stream) {
  if (!cam) return fail(RTA_E_INVALID_ARG, "null camera");
  if (!rta::extractor_supported(extractor)) return fail(RTA_E_INVALID_ARG, "unknown extractor");
  if (n_evt < 0) return fail(RTA_E_INVALID_ARG, "negative event count");
  if (n_evt > 0x7fffffffLL) return fail(RTA_E_SHAPE, "too many events for one launch");
  if (n_evt == 0) return RTA_OK;
  if (!traces || !aligned16(traces)) return fail(RTA_E_INVALID_ARG, "traces must be non-null and 16-byte aligned");
  RTA_HIP(rta::launch_calibrate(cam->dev, extractor, traces, n_evt, S, D, sstar, peak, gain, q, t,
                                (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_clean(const rta_camera* cam, const rta_clean_params* levels, const int32_t* D, const uint8_t* gain,
                     int64_t n_evt, uint8_t* mask, rta_stream stream) {
  if (!cam) return fail(RTA_E_INVALID_ARG, "null camera");
  if (levels) {
    if (!std::isfinite(levels->t_pic) || !std::isfinite(levels->t_bnd) || levels->t_bnd > levels->t_pic)
      return fail(RTA_E_INVALID_ARG, "cleaning levels must be finite with t_bnd <= t_pic");
    const double m = 256.0 * cam->max_a;
    if (std::fabs(m * (double)levels->t_pic) > 2.0e9 || std::fabs(m * (double)levels->t_bnd) > 2.0e9)
      return fail(RTA_E_INVALID_ARG, "threshold overflow");
  }
  if (n_evt < 0) return fail(RTA_E_INVALID_ARG, "negative event count");
  if (n_evt > 0x7fffffffLL) return fail(RTA_E_SHAPE, "too many events for one launch");
  if (n_evt == 0) return RTA_OK;
  if (!D || !mask) return fail(RTA_E_INVALID_ARG, "null D or mask");
  RTA_HIP(rta::launch_clean(cam->dev, levels, D, gain, n_evt, mask, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_hillas(const rta_camera* cam, const float* q_pe, const float* t, const uint8_t* mask,
                      const uint8_t* gain, int64_t n_evt, rta_hillas_rec* out, rta_stream stream) {
  if (!cam) return fail(RTA_E_INVALID_ARG, "null camera");
  if (n_evt < 0) return fail(RTA_E_INVALID_ARG, "negative event count");
  if (n_evt > 0x7fffffffLL) return fail(RTA_E_SHAPE, "too many events for one launch");
  if (n_evt == 0) return RTA_OK;
  if (!q_pe || !t || !mask || !out) return fail(RTA_E_INVALID_ARG, "null q_pe, t, mask or output");
  RTA_HIP(rta::launch_hillas(cam->dev, q_pe, nullptr, t, mask, gain, n_evt, out, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_hillas_q8(const rta_camera* cam, const int32_t* D, const float* t, const uint8_t* mask,
                         const uint8_t* gain, int64_t n_evt, rta_hillas_rec* out, rta_stream stream) {
  if (!cam) return fail(RTA_E_INVALID_ARG, "null camera");
  if (n_evt < 0) return fail(RTA_E_INVALID_ARG, "negative event count");
  if (n_evt > 0x7fffffffLL) return fail(RTA_E_SHAPE, "too many events for one launch");
  if (n_evt == 0) return RTA_OK;
  if (!D || !t || !mask || !out) return fail(RTA_E_INVALID_ARG, "null D, t, mask or output");
  RTA_HIP(rta::launch_hillas(cam->dev, nullptr, D, t, mask, gain, n_evt, out, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_pipeline_create(rta_camera* const* cams, int32_t n_types, const rta_pipeline_params* params,
                               rta_pipeline** out) {
  if (!out) return fail(RTA_E_INVALID_ARG, "null output handle");
  *out = nullptr;
  if (!cams || !params || n_types < 1 || n_types > RTA_MAX_TYPES)
    return fail(RTA_E_INVALID_ARG, "need 1..RTA_MAX_TYPES camera handles and params");
  for (int i = 0; i < n_types; ++i)
    if (!cams[i]) return fail(RTA_E_INVALID_ARG, "null camera handle");
  for (int i = 1; i < n_types; ++i)
    if (cams[i]->dev.window != cams[0]->dev.window) return fail(RTA_E_SHAPE, "all camera types need one window");
  if (!rta::extractor_supported(params->extractor)) return fail(RTA_E_INVALID_ARG, "unknown extractor");
  if (params->do_stereo && (!(params->max_width_ratio > 0.f) || !(params->max_cond > 1.f)))
    return fail(RTA_E_INVALID_ARG, "stereo cuts must be positive");
  rta_pipeline* p = new (std::nothrow) rta_pipeline();
  if (!p) return fail(RTA_E_NOMEM, "host allocation failed");
  p->cams.assign(cams, cams + n_types);
  p->params = *params;
  p->window = cams[0]->dev.window;
  p->sched = rta_schedule{8, 4, 0, 8};
  if (hipGetDevice(&p->device) != hipSuccess ||
      hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) {
    delete p;
    return fail(RTA_E_HIP, "device query failed");
  }
  void* mem = nullptr;
  if (hipMalloc(&mem, 256) != hipSuccess) {
    delete p;
    return fail(RTA_E_NOMEM, "device allocation failed");
  }
  p->d_queue = static_cast<unsigned long long*>(mem);
  p->d_status = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(mem) + 64);
  if (hipMemset(mem, 0, 256) != hipSuccess ||
      hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipFree(mem);
    delete p;
    return fail(RTA_E_HIP, "pipeline initialisation failed");
  }
  p->params.tune_cache = nullptr;  // the caller's string is not kept
  p->params.mlp = nullptr;         // kept as the attached network below
  p->params.boxcut = nullptr;
  if (params->mlp || params->boxcut) {
    rta_status as = (params->mlp && params->boxcut)
                        ? rta_pipeline_attach_mlp(p, params->mlp, params->boxcut)
                        : fail(RTA_E_INVALID_ARG, "a network needs its box-cut tables and the reverse");
    if (as != RTA_OK) {
      const std::string why = g_err;
      (void)rta_pipeline_destroy(p);
      return fail(as, why);
    }
  }
  rta_status ks = make_tune_key(p, &p->tune_key);
  if (ks != RTA_OK) {
    (void)rta_pipeline_destroy(p);
    return ks;
  }
  if (params->tune_cache) {
    p->tune_cache = params->tune_cache;
    rta_schedule cached{};
    if (rta_tune_cache_lookup(params->tune_cache, p->tune_key.c_str(), &cached, nullptr) == RTA_OK)
      p->sched = cached;
    else
      p->untuned = true;
    g_err.clear();
  }
  *out = p;
  return RTA_OK;
}

rta_status rta_pipeline_destroy(rta_pipeline* p) {
  if (!p) return RTA_OK;
  (void)hipDeviceSynchronize();
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->d_queue) (void)hipFree(p->d_queue);
  delete p;
  return RTA_OK;
}

rta_status rta_set_schedule(rta_pipeline* p, const rta_schedule* s) {
  if (!p || !s) return fail(RTA_E_INVALID_ARG, "null pipeline or schedule");
  if (!rta::schedule_supported(*s)) return fail(RTA_E_UNSUPPORTED, "schedule not compiled");
  p->sched = *s;
  p->untuned = false;
  return RTA_OK;
}

rta_status rta_get_schedule(const rta_pipeline* p, rta_schedule* s) {
  if (!p || !s) return fail(RTA_E_INVALID_ARG, "null pipeline or schedule");
  *s = p->sched;
  return RTA_OK;
}

rta_status rta_list_schedules(rta_schedule* out, int32_t cap, int32_t* n) {
  if (!n || cap < 0 || (cap > 0 && !out)) return fail(RTA_E_INVALID_ARG, "bad schedule list arguments");
  *n = rta::list_schedules(out, cap);
  return RTA_OK;
}

rta_status rta_pipeline_tune_key(const rta_pipeline* p, char* key, int32_t cap) {
  if (!p || !key || cap <= 0) return fail(RTA_E_INVALID_ARG, "null pipeline or key buffer");
  if ((int64_t)p->tune_key.size() + 1 > cap) return fail(RTA_E_INVALID_ARG, "key buffer too small");
  std::memcpy(key, p->tune_key.c_str(), p->tune_key.size() + 1);
  return RTA_OK;
}

rta_status rta_tune_cache_lookup(const char* path, const char* key, rta_schedule* s, float* ms) {
  if (!path || !key || !s) return fail(RTA_E_INVALID_ARG, "null path, key or schedule");
  std::vector<std::string> lines;
  {
    std::lock_guard<std::mutex> lk(g_tune_file_mu);
    if (!read_lines(path, &lines)) return fail(RTA_E_UNTUNED, std::string("no tune cache at ") + path);
  }
  std::string k;
  rta_schedule v{};
  float t = 0.f;
  for (const std::string& line : lines) {
    if (!parse_tune_line(line, &k, &v, &t) || k != key) continue;
    if (!rta::schedule_supported(v)) return fail(RTA_E_UNTUNED, "cached schedule is not compiled into this library");
    *s = v;
    if (ms) *ms = t;
    return RTA_OK;
  }
  return fail(RTA_E_UNTUNED, std::string("no tune cache entry for ") + key);
}

rta_status rta_tune_cache_store(const char* path, const char* key, const rta_schedule* s, float ms) {
  if (!path || !key || !s || !*key) return fail(RTA_E_INVALID_ARG, "null path, key or schedule");
  if (std::strpbrk(key, "\t\r\n")) return fail(RTA_E_INVALID_ARG, "tune keys may not hold tabs or line breaks");
  if (!rta::schedule_supported(*s)) return fail(RTA_E_UNSUPPORTED, "schedule not compiled");
  std::lock_guard<std::mutex> lk(g_tune_file_mu);
  std::vector<std::string> lines, kept;
  (void)read_lines(path, &lines);  // a missing file starts empty
  kept.push_back("# rta schedule tune cache: key<TAB>pix_per_lane waves_per_wg wg_per_cu chunk<TAB>ms");
  std::string k;
  rta_schedule v{};
  float t = 0.f;
  for (const std::string& line : lines)
    if (parse_tune_line(line, &k, &v, &t) && k != key) kept.push_back(line);
  char buf[128];
  std::snprintf(buf, sizeof(buf), "\t%d %d %d %d\t%.6g", (int)s->pix_per_lane, (int)s->waves_per_wg,
                (int)s->wg_per_cu, (int)s->chunk, (double)ms);
  kept.push_back(std::string(key) + buf);
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return fail(RTA_E_INVALID_ARG, "cannot write " + tmp + ": " + std::strerror(errno));
  bool ok = true;
  for (const std::string& line : kept) ok = ok && std::fprintf(f, "%s\n", line.c_str()) > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    const std::string why = std::strerror(errno);
    (void)std::remove(tmp.c_str());
    return fail(RTA_E_INVALID_ARG, "cannot write tune cache " + std::string(path) + ": " + why);
  }
  return RTA_OK;
}

rta_status rta_pipeline_tune(rta_pipeline* p, const rta_batch* batch, rta_hillas_rec* tel_out,
                             rta_event_rec* evt_out, const rta_schedule* cands, int32_t n_cands, int32_t reps,
                             float* ms, rta_schedule* best, rta_stream stream) {
  rta_status s = check_batch(p, batch, tel_out, evt_out, false);
  if (s != RTA_OK) return s;
  if (reps < 1 || reps > 100) return fail(RTA_E_INVALID_ARG, "reps must be in 1..100");
  std::vector<rta_schedule> list;
  if (cands) {
    if (n_cands < 1) return fail(RTA_E_INVALID_ARG, "need at least one candidate schedule");
    list.assign(cands, cands + n_cands);
  } else {
    list.resize(rta::list_schedules(nullptr, 0));
    list.resize(rta::list_schedules(list.data(), (int)list.size()));
  }
  for (const rta_schedule& c : list)
    if (!rta::schedule_supported(c)) return fail(RTA_E_UNSUPPORTED, "candidate schedule not compiled");
  const hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  RTA_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(RTA_E_HIP, "hipEventCreate failed");
  }
  const rta_schedule prev = p->sched;
  std::vector<float> med(list.size(), 0.f), t(reps);
  rta_status err = RTA_OK;
  for (size_t i = 0; i < list.size() && err == RTA_OK; ++i) {
    p->sched = list[i];
    err = launch_batch(p, batch, tel_out, evt_out, p->d_queue, p->d_status, st);
    for (int r = 0; r < reps && err == RTA_OK; ++r) {
      hipError_t e = hipEventRecord(e0, st);
      if (e == hipSuccess) err = launch_batch(p, batch, tel_out, evt_out, p->d_queue, p->d_status, st);
      if (e == hipSuccess && err == RTA_OK) e = hipEventRecord(e1, st);
      if (e == hipSuccess && err == RTA_OK) e = hipEventSynchronize(e1);
      if (e == hipSuccess && err == RTA_OK) e = hipEventElapsedTime(&t[r], e0, e1);
      if (e != hipSuccess && err == RTA_OK)
        err = fail(RTA_E_HIP, std::string("timing a schedule: ") + hipGetErrorString(e));
    }
    if (err == RTA_OK) {
      std::sort(t.begin(), t.end());
      med[i] = t[reps / 2];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != RTA_OK) {
    p->sched = prev;
    return err;
  }
  size_t k = 0;
  for (size_t i = 1; i < list.size(); ++i)
    if (med[i] < med[k]) k = i;
  p->sched = list[k];
  p->untuned = false;
  if (ms) std::copy(med.begin(), med.end(), ms);
  if (best) *best = list[k];
  if (!p->tune_cache.empty())
    return rta_tune_cache_store(p->tune_cache.c_str(), p->tune_key.c_str(), &list[k], med[k]);
  return RTA_OK;
}

rta_status rta_process_batch(rta_pipeline* pipe, const rta_batch* batch, rta_hillas_rec* tel_out,
                             rta_event_rec* evt_out, rta_stream stream) {
  rta_status s = check_batch(pipe, batch, tel_out, evt_out);
  if (s != RTA_OK) return s;
  return launch_batch(pipe, batch, tel_out, evt_out, pipe->d_queue, pipe->d_status, (hipStream_t)stream);
}

rta_status rta_process_batch_noalloc(const rta_pipeline* pipe, const rta_batch* batch, rta_hillas_rec* tel_out,
                                     rta_event_rec* evt_out, uint32_t* status_out, rta_stream stream) {
  rta_status s = check_batch(pipe, batch, tel_out, evt_out);
  if (s != RTA_OK) return s;
  int dev = -1;
  RTA_HIP(hipGetDevice(&dev));
  if (dev != pipe->device) return fail(RTA_E_INVALID_ARG, "the pipeline's device must be the current device");
  uint8_t* base = nullptr;
  s = noalloc_scratch(dev, &base);
  if (s != RTA_OK) return s;
  unsigned long long* queue = reinterpret_cast<unsigned long long*>(base + kScratchQueue);
  uint32_t* status = reinterpret_cast<uint32_t*>(base + kScratchStatus);
  const hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_scratch_reset, dim3(1), dim3(64), 0, st, queue, status);
  RTA_HIP(hipGetLastError());
  s = launch_batch(pipe, batch, tel_out, evt_out, queue, status, st);
  if (s != RTA_OK) return s;
  if (status_out) {
    hipLaunchKernelGGL(k_status_copy, dim3(1), dim3(64), 0, st, (const uint32_t*)status, status_out);
    RTA_HIP(hipGetLastError());
  }
  return RTA_OK;
}

rta_status rta_stereo(rta_pipeline* pipe, const int64_t* evt_tel_off, const int32_t* tel_type, int64_t n_evt,
                      int64_t n_tel, const rta_hillas_rec* tel, rta_event_rec* evt_out, rta_stream stream) {
  if (!pipe) return fail(RTA_E_INVALID_ARG, "null pipeline");
  if (n_evt < 0 || n_tel < 0) return fail(RTA_E_INVALID_ARG, "negative count");
  if (n_evt == 0) return RTA_OK;
  if (!evt_tel_off || !evt_out || (n_tel > 0 && (!tel_type || !tel))) return fail(RTA_E_INVALID_ARG, "null pointer");
  rta::EventArgs ea;
  fill_event_args(pipe, ea);
  ea.evt_tel_off = evt_tel_off;
  ea.tel_type = tel_type;
  ea.n_evt = n_evt;
  ea.n_tel = n_tel;
  ea.tel = const_cast<rta_hillas_rec*>(tel);
  ea.out = evt_out;
  ea.status = pipe->d_status;
  RTA_HIP(rta::launch_event(ea, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_batch_status(rta_pipeline* p, uint32_t* status) {
  if (!p || !status) return fail(RTA_E_INVALID_ARG, "null pipeline or status");
  RTA_HIP(hipDeviceSynchronize());
  RTA_HIP(hipMemcpy(status, p->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost));
  RTA_HIP(hipMemset(p->d_status, 0, sizeof(uint32_t)));
  RTA_HIP(hipDeviceSynchronize());
  return RTA_OK;
}

rta_status rta_frame_packets(const rta_camera_info* types, int32_t n_types, const uint8_t* bytes, int64_t n_bytes,
                             int64_t cap, int64_t* pkt_off, int32_t* tel_type, int64_t* tel_trace_off,
                             int64_t* n_pkt, int64_t* pool_elems, int64_t* consumed) {
  if (!n_pkt || !pool_elems || !consumed) return fail(RTA_E_INVALID_ARG, "null count output");
  *n_pkt = *pool_elems = *consumed = 0;
  if (n_types < 0 || n_types > RTA_MAX_TYPES || (n_types > 0 && !types)) return fail(RTA_E_INVALID_ARG, "bad types");
  if (n_bytes < 0 || cap < 0 || (n_bytes > 0 && !bytes) || (cap > 0 && (!pkt_off || !tel_type || !tel_trace_off)))
    return fail(RTA_E_INVALID_ARG, "null or negative argument");
  auto u16 = [&](int64_t o) { return (uint32_t)bytes[o] << 8 | bytes[o + 1]; };
  int64_t pos = 0, n = 0, pool = 0;
  while (pos + 8 <= n_bytes && n < cap) {
    const int64_t total = (int64_t)((u16(pos + 4) << 16) | u16(pos + 6)) + 9;
    if (total < 34) {
      *n_pkt = n;
      *pool_elems = pool;
      *consumed = pos;
      return fail(RTA_E_SHAPE, "packet framing lost (data length below the smallest packet)");
    }
    if (pos + total > n_bytes) break;
    const int ty = bytes[pos + 11];
    const int N = (int)u16(pos + 18), T = (int)u16(pos + 20), G = bytes[pos + 22];
    pkt_off[n] = pos;
    if (ty < n_types && types[ty].n_pix == N && types[ty].n_samp == T && types[ty].n_gain == G) {
      tel_type[n] = ty;
      tel_trace_off[n] = pool;
      pool += types[ty].event_elems;
    } else {
      tel_type[n] = -1;
      tel_trace_off[n] = 0;
    }
    ++n;
    pos += total;
  }
  *n_pkt = n;
  *pool_elems = pool;
  *consumed = pos;
  return RTA_OK;
}

rta_status rta_decode_packets(rta_pipeline* pipe, const uint8_t* bytes, int64_t n_bytes, const int64_t* pkt_off,
                              int32_t* tel_type, const int64_t* tel_trace_off, int64_t n_pkt, uint16_t* pool,
                              int64_t pool_elems, rta_packet_rec* rec, rta_stream stream) {
  if (!pipe) return fail(RTA_E_INVALID_ARG, "null pipeline");
  if (n_pkt < 0 || n_bytes < 0 || pool_elems < 0) return fail(RTA_E_INVALID_ARG, "negative size");
  if (n_pkt == 0) return RTA_OK;
  if (n_pkt > 0x7fffffffLL) return fail(RTA_E_SHAPE, "too many packets for one launch");
  if (!bytes || !pkt_off || !tel_type || !tel_trace_off || (pool_elems > 0 && !pool))
    return fail(RTA_E_INVALID_ARG, "null pointer");
  if (!aligned16(bytes) || (pool && !aligned16(pool))) return fail(RTA_E_INVALID_ARG, "bytes and pool must be 16-byte aligned");
  rta::DecodeArgs da;
  std::memset(&da, 0, sizeof(da));
  for (size_t i = 0; i < pipe->cams.size(); ++i) da.cams[i] = pipe->cams[i]->dev;
  da.n_types = (int32_t)pipe->cams.size();
  da.bytes = bytes;
  da.n_bytes = n_bytes;
  da.pkt_off = pkt_off;
  da.tel_type = tel_type;
  da.tel_trace_off = tel_trace_off;
  da.n_pkt = n_pkt;
  da.pool = pool;
  da.pool_elems = pool_elems;
  da.rec = rec;
  da.status = pipe->d_status;
  RTA_HIP(rta::launch_decode(da, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_health(rta_camera* cam, const uint16_t* traces, int64_t n_evt, const rta_health_params* params,
                      rta_pixel_health* pix, rta_camera_health* out, rta_stream stream) {
  if (!cam || !params) return fail(RTA_E_INVALID_ARG, "null camera or parameters");
  if (n_evt < 1) return fail(RTA_E_INVALID_ARG, "n_evt must be >= 1");
  if (n_evt > 0x7fffffffLL) return fail(RTA_E_SHAPE, "too many events for one launch");
  if (!traces || !aligned16(traces)) return fail(RTA_E_INVALID_ARG, "traces must be non-null and 16-byte aligned");
  if (!pix || !out) return fail(RTA_E_INVALID_ARG, "null outputs");
  const float v[5] = {params->rms_dead, params->noisy_factor, params->ped_tol, params->sat_frac,
                      params->bad_frac_max};
  for (float x : v)
    if (!std::isfinite(x)) return fail(RTA_E_INVALID_ARG, "health thresholds must be finite");
  RTA_HIP(rta::launch_health(cam->dev, traces, n_evt, *params, cam->health_part, cam->health_acc, pix, out,
                             (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_sam_create(const rta_sam_params* p, rta_sam** out) {
  if (!p || !out) return fail(RTA_E_INVALID_ARG, "null parameters or output handle");
  *out = nullptr;
  if (p->grid < 1 || p->grid > RTA_SAM_MAX_GRID) return fail(RTA_E_SHAPE, "grid must be in [1, RTA_SAM_MAX_GRID]");
  if (p->n_bins < 1) return fail(RTA_E_SHAPE, "n_bins must be >= 1");
  if ((int64_t)p->n_bins * p->grid * p->grid > 0x7fffffffLL) return fail(RTA_E_SHAPE, "counts cube too large");
  if (!(p->bin_s > 0.0) || !std::isfinite(p->t0) || !std::isfinite(p->bin_s))
    return fail(RTA_E_INVALID_ARG, "bin_s must be > 0 and t0 finite");
  if (!(p->cell > 0.f) || !std::isfinite(p->cell)) return fail(RTA_E_INVALID_ARG, "cell must be > 0");
  if (!(p->r_on >= 0.f && p->r_on < p->r_in && p->r_in < p->r_out && p->r_out <= (float)RTA_SAM_MAX_REACH))
    return fail(RTA_E_INVALID_ARG, "radii must satisfy 0 <= r_on < r_in < r_out <= RTA_SAM_MAX_REACH");
  if (!std::isfinite(p->gamma_cut) || !std::isfinite(p->sigma_alert))
    return fail(RTA_E_INVALID_ARG, "cuts must be finite");
  if (p->n_scales < 1 || p->n_scales > RTA_SAM_MAX_SCALES) return fail(RTA_E_SHAPE, "n_scales out of range");
  for (int k = 0; k < p->n_scales; ++k)
    if (p->scales[k] < 1 || p->scales[k] > p->n_bins) return fail(RTA_E_SHAPE, "scale must be in [1, n_bins]");
  // disc and ring offsets, classified in FP64 from the float radii
  std::vector<int32_t> offs;
  const double on2 = (double)p->r_on * p->r_on, in2 = (double)p->r_in * p->r_in, out2 = (double)p->r_out * p->r_out;
  const int reach = (int)std::ceil(p->r_out);
  for (int dy = -reach; dy <= reach; ++dy)
    for (int dx = -reach; dx <= reach; ++dx) {
      const double d2 = (double)(dx * dx + dy * dy);
      const int kind = d2 <= on2 ? 1 : (d2 > in2 && d2 <= out2 ? 2 : 0);
      if (kind) offs.push_back((dx + 128) | ((dy + 128) << 8) | (kind << 16));
    }
  const size_t G2 = (size_t)p->grid * p->grid;
  const size_t oC = 0, oW = round256((size_t)p->n_bins * G2 * 4), oO = oW + round256((size_t)p->n_scales * G2 * 4);
  const size_t total = oO + round256(offs.size() * 4);
  rta_sam* sam = new (std::nothrow) rta_sam();
  if (!sam) return fail(RTA_E_NOMEM, "host allocation failed");
  if (hipGetDevice(&sam->device) != hipSuccess || hipMalloc(&sam->dmem, total) != hipSuccess) {
    delete sam;
    return fail(RTA_E_NOMEM, "device allocation for the monitor failed");
  }
  uint8_t* base = static_cast<uint8_t*>(sam->dmem);
  if (hipMemcpy(base + oO, offs.data(), offs.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(sam->dmem);
    delete sam;
    return fail(RTA_E_HIP, "copy of the offset table failed");
  }
  rta::SamDev& d = sam->dev;
  d.grid = p->grid;
  d.n_bins = p->n_bins;
  d.n_scales = p->n_scales;
  d.n_offs = (int32_t)offs.size();
  d.t0 = p->t0;
  d.bin_s = p->bin_s;
  d.cell = p->cell;
  d.gamma_cut = p->gamma_cut;
  d.sigma_alert = p->sigma_alert;
  d.r_on2 = (float)on2;
  for (int k = 0; k < RTA_SAM_MAX_SCALES; ++k) d.scales[k] = k < p->n_scales ? p->scales[k] : 1;
  d.counts = reinterpret_cast<int32_t*>(base + oC);
  d.win = reinterpret_cast<int32_t*>(base + oW);
  d.offs = reinterpret_cast<const int32_t*>(base + oO);
  if (rta::launch_sam_clear(d, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(sam->dmem);
    delete sam;
    return fail(RTA_E_HIP, "clearing the counts failed");
  }
  *out = sam;
  return RTA_OK;
}

rta_status rta_sam_destroy(rta_sam* sam) {
  if (!sam) return RTA_OK;
  if (sam->dmem) (void)hipFree(sam->dmem);
  delete sam;
  return RTA_OK;
}

rta_status rta_sam_clear(rta_sam* sam, rta_stream stream) {
  if (!sam) return fail(RTA_E_INVALID_ARG, "null monitor");
  RTA_HIP(rta::launch_sam_clear(sam->dev, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_sam_fill(rta_sam* sam, const rta_event_rec* evt, const double* t, int64_t n, rta_stream stream) {
  if (!sam) return fail(RTA_E_INVALID_ARG, "null monitor");
  if (n < 0) return fail(RTA_E_INVALID_ARG, "negative event count");
  if (n == 0) return RTA_OK;
  if (n > 0x7fffffffLL * 256) return fail(RTA_E_SHAPE, "too many events for one launch");
  if (!evt || !t) return fail(RTA_E_INVALID_ARG, "null events or times");
  RTA_HIP(rta::launch_sam_fill(sam->dev, evt, t, n, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_sam_search(rta_sam* sam, int32_t end_bin, double* significance, int32_t* n_on, int32_t* n_off,
                          rta_sam_alert* alerts, int32_t max_alerts, int32_t* n_alerts, rta_stream stream) {
  if (!sam) return fail(RTA_E_INVALID_ARG, "null monitor");
  if (end_bin < 0 || end_bin >= sam->dev.n_bins) return fail(RTA_E_INVALID_ARG, "end_bin out of range");
  if (max_alerts < 0 || (max_alerts > 0 && !alerts) || !n_alerts)
    return fail(RTA_E_INVALID_ARG, "null alert outputs");
  RTA_HIP(rta::launch_sam_search(sam->dev, end_bin, significance, n_on, n_off, alerts, max_alerts, n_alerts,
                                 (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_sam_counts(const rta_sam* sam, int32_t* dst, rta_stream stream) {
  if (!sam || !dst) return fail(RTA_E_INVALID_ARG, "null monitor or output");
  const size_t bytes = (size_t)sam->dev.n_bins * sam->dev.grid * sam->dev.grid * 4;
  RTA_HIP(hipMemcpyAsync(dst, sam->dev.counts, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_graph_capture(rta_pipeline* pipe, const rta_batch* batch, rta_hillas_rec* tel_out,
                             rta_event_rec* evt_out, rta_graph** out) {
  if (!out) return fail(RTA_E_INVALID_ARG, "null output handle");
  *out = nullptr;
  rta_status s = check_batch(pipe, batch, tel_out, evt_out);
  if (s != RTA_OK) return s;
  rta_graph* g = new (std::nothrow) rta_graph();
  if (!g) return fail(RTA_E_NOMEM, "host allocation failed");
  hipError_t e = hipStreamBeginCapture(pipe->capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete g;
    return fail(RTA_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  s = launch_batch(pipe, batch, tel_out, evt_out, pipe->d_queue, pipe->d_status, pipe->capture_stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(pipe->capture_stream, &graph);
  if (s != RTA_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    delete g;
    return s != RTA_OK ? s : fail(RTA_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete g;
    return fail(RTA_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  g->graph = graph;
  *out = g;
  return RTA_OK;
}

rta_status rta_graph_launch(rta_graph* g, rta_stream stream) {
  if (!g || !g->exec) return fail(RTA_E_INVALID_ARG, "null graph");
  RTA_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_graph_destroy(rta_graph* g) {
  if (!g) return RTA_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return RTA_OK;
}

static bool boxcut_valid(const rta_boxcut_desc* bc) {
  if (!bc || bc->n_bins < 1 || bc->n_bins > RTA_BOXCUT_MAX_BINS) return false;
  if (!std::isfinite(bc->lgs_lo) || !std::isfinite(bc->lgs_hi) || !(bc->lgs_hi > bc->lgs_lo)) return false;
  for (int b = 0; b < bc->n_bins; ++b)
    if (!std::isfinite(bc->w_mean[b]) || !std::isfinite(bc->l_mean[b]) || !(bc->w_std[b] > 0.f) ||
        !(bc->l_std[b] > 0.f))
      return false;
  for (int f = 0; f < RTA_MLP_N_FEATURES; ++f)
    if (std::isnan(bc->feat_lo[f]) || std::isnan(bc->feat_hi[f])) return false;
  return std::isfinite(bc->e_a) && std::isfinite(bc->e_b) && !std::isnan(bc->cut_w) && !std::isnan(bc->cut_l);
}

rta_status rta_features(const rta_hillas_rec* rec, int64_t n, float* x, rta_stream stream) {
  if (n < 0) return fail(RTA_E_INVALID_ARG, "negative count");
  if (n == 0) return RTA_OK;
  if (!rec || !x) return fail(RTA_E_INVALID_ARG, "null pointer");
  if ((n + 255) / 256 > 0x7fffffffLL) return fail(RTA_E_SHAPE, "too many records for one launch");
  RTA_HIP(rta::launch_features(rec, n, x, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_classify(rta_mlp* m, const rta_boxcut_desc* bc, const rta_hillas_rec* rec, int64_t n, float* out,
                        rta_stream stream) {
  if (!boxcut_valid(bc)) return fail(RTA_E_INVALID_ARG, "invalid box-cut tables");
  if (m && !m->has_params) return fail(RTA_E_INVALID_ARG, "network parameters not set");
  if (n < 0) return fail(RTA_E_INVALID_ARG, "negative count");
  if (n == 0) return RTA_OK;
  if (!rec || !out) return fail(RTA_E_INVALID_ARG, "null pointer");
  if ((n + 63) / 64 > 0x7fffffffLL) return fail(RTA_E_SHAPE, "too many records for one launch");
  rta::MlpDev none{};
  RTA_HIP(rta::launch_classify(m ? m->dev : none, m != nullptr, *bc, rec, n, out, (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_pipeline_attach_mlp(rta_pipeline* pipe, rta_mlp* m, const rta_boxcut_desc* bc) {
  if (!pipe) return fail(RTA_E_INVALID_ARG, "null pipeline");
  if (!m) {
    pipe->mlp = nullptr;
    pipe->have_box = false;
    return RTA_OK;
  }
  if (!m->has_params) return fail(RTA_E_INVALID_ARG, "network parameters not set");
  if (!boxcut_valid(bc)) return fail(RTA_E_INVALID_ARG, "invalid box-cut tables");
  pipe->mlp = m;
  pipe->bc = *bc;
  pipe->have_box = true;
  return RTA_OK;
}

rta_status rta_mlp_create(const rta_mlp_desc* d, rta_mlp** out) {
  if (!d || !out) return fail(RTA_E_INVALID_ARG, "null descriptor or output handle");
  *out = nullptr;
  if (d->max_batch < 1 || d->max_batch > (1 << 22)) return fail(RTA_E_SHAPE, "max_batch must be in [1, 2^22]");
  if (!(d->lr > 0.f) || !(d->beta1 >= 0.f && d->beta1 < 1.f) || !(d->beta2 >= 0.f && d->beta2 < 1.f) ||
      !(d->eps > 0.f))
    return fail(RTA_E_INVALID_ARG, "bad Adam hyper-parameters");
  rta_mlp* m = new (std::nothrow) rta_mlp();
  if (!m) return fail(RTA_E_NOMEM, "host allocation failed");
  m->max_batch = d->max_batch;
  m->bpad_max = (d->max_batch + 63) & ~63;
  m->lr = d->lr; m->beta1 = d->beta1; m->beta2 = d->beta2; m->eps = d->eps;
  const size_t P = rta::kNParams, Bp = (size_t)m->bpad_max;
  // sub-array byte sizes, each rounded to 256
  const size_t sizes[] = {P * 4, P * 4, P * 4, P * 4,                       // master m1 m2 grad
                          rta::kGradSplit * P * 4,                          // gpart
                          64 * 16 * 2, 64 * 64 * 2, 64 * 64 * 2, 16 * 64 * 2,  // W1t..W4t
                          64 * 64 * 2, 64 * 64 * 2, 64 * 16 * 2,             // W2n..W4n
                          64 * 4, 64 * 4, 64 * 4, 16 * 4, 16 * 4, 16 * 4,     // b1..b4 mean std
                          16 * Bp * 2, 64 * Bp * 2, 64 * Bp * 2, 64 * Bp * 2,  // H0..H3
                          64 * Bp * 2, 64 * Bp * 2, 64 * Bp * 2, 16 * Bp * 2,  // G1..G4
                          (Bp + 1) * 4};
  const int n = sizeof(sizes) / sizeof(sizes[0]);
  size_t off[32], total = 0;
  for (int i = 0; i < n; ++i) { off[i] = total; total += round256(sizes[i]); }
  if (hipMalloc(&m->dmem, total) != hipSuccess) {
    delete m;
    return fail(RTA_E_NOMEM, "device allocation for the network failed");
  }
  if (hipMemset(m->dmem, 0, total) != hipSuccess) {
    (void)hipFree(m->dmem);
    delete m;
    return fail(RTA_E_HIP, "clearing network memory failed");
  }
  uint8_t* b = static_cast<uint8_t*>(m->dmem);
  rta::MlpDev& w = m->dev;
  int i = 0;
  w.master = (float*)(b + off[i++]); w.m1 = (float*)(b + off[i++]); w.m2 = (float*)(b + off[i++]);
  w.grad = (float*)(b + off[i++]);
  w.gpart = (float*)(b + off[i++]);
  w.W1t = (uint16_t*)(b + off[i++]); w.W2t = (uint16_t*)(b + off[i++]); w.W3t = (uint16_t*)(b + off[i++]);
  w.W4t = (uint16_t*)(b + off[i++]);
  w.W2n = (uint16_t*)(b + off[i++]); w.W3n = (uint16_t*)(b + off[i++]); w.W4n = (uint16_t*)(b + off[i++]);
  w.b1 = (float*)(b + off[i++]); w.b2 = (float*)(b + off[i++]); w.b3 = (float*)(b + off[i++]);
  w.b4 = (float*)(b + off[i++]); w.mean = (float*)(b + off[i++]); w.stdv = (float*)(b + off[i++]);
  w.H0 = (uint16_t*)(b + off[i++]); w.H1 = (uint16_t*)(b + off[i++]); w.H2 = (uint16_t*)(b + off[i++]);
  w.H3 = (uint16_t*)(b + off[i++]);
  w.G1 = (uint16_t*)(b + off[i++]); w.G2 = (uint16_t*)(b + off[i++]); w.G3 = (uint16_t*)(b + off[i++]);
  w.G4 = (uint16_t*)(b + off[i++]);
  w.loss_row = (float*)(b + off[i++]);
  *out = m;
  return RTA_OK;
}

rta_status rta_mlp_destroy(rta_mlp* m) {
  if (!m) return RTA_OK;
  if (m->dmem) (void)hipFree(m->dmem);
  delete m;
  return RTA_OK;
}

rta_status rta_mlp_set_params(rta_mlp* m, const float* params, const float* mean, const float* stdv) {
  if (!m || !params || !mean || !stdv) return fail(RTA_E_INVALID_ARG, "null argument");
  for (int k = 0; k < rta::kNParams; ++k)
    if (!std::isfinite(params[k])) return fail(RTA_E_INVALID_ARG, "non-finite parameter");
  float mu[16] = {0}, sd[16];
  for (int k = 0; k < 16; ++k) sd[k] = 1.f;
  for (int k = 0; k < RTA_MLP_N_FEATURES; ++k) {
    if (!std::isfinite(mean[k]) || !std::isfinite(stdv[k]) || !(stdv[k] > 0.f))
      return fail(RTA_E_INVALID_ARG, "feature mean / std must be finite with std > 0");
    mu[k] = mean[k];
    sd[k] = stdv[k];
  }
  RTA_HIP(hipMemcpy(m->dev.master, params, sizeof(float) * rta::kNParams, hipMemcpyHostToDevice));
  RTA_HIP(hipMemset(m->dev.m1, 0, sizeof(float) * rta::kNParams));
  RTA_HIP(hipMemset(m->dev.m2, 0, sizeof(float) * rta::kNParams));
  RTA_HIP(hipMemcpy(m->dev.mean, mu, sizeof(mu), hipMemcpyHostToDevice));
  RTA_HIP(hipMemcpy(m->dev.stdv, sd, sizeof(sd), hipMemcpyHostToDevice));
  RTA_HIP(rta::launch_mlp_adam(m->dev, false, 0.f, 0.f, 0.f, 1.f, 1.f, 1.f, nullptr));
  RTA_HIP(hipDeviceSynchronize());
  m->step = 0;
  m->has_params = true;
  return RTA_OK;
}

rta_status rta_mlp_get_params(rta_mlp* m, float* params) {
  if (!m || !params) return fail(RTA_E_INVALID_ARG, "null argument");
  RTA_HIP(hipDeviceSynchronize());
  RTA_HIP(hipMemcpy(params, m->dev.master, sizeof(float) * rta::kNParams, hipMemcpyDeviceToHost));
  return RTA_OK;
}

rta_status rta_mlp_forward(rta_mlp* m, const float* x, int64_t B, float* out, rta_stream stream) {
  if (!m) return fail(RTA_E_INVALID_ARG, "null network");
  if (!m->has_params) return fail(RTA_E_INVALID_ARG, "network parameters not set");
  if (B < 0 || B > 0x7fffffffLL - 64) return fail(RTA_E_SHAPE, "bad batch size");
  if (B == 0) return RTA_OK;
  if (!x || !out) return fail(RTA_E_INVALID_ARG, "null input or output");
  const int Bpad = (int)((B + 63) & ~63LL);
  RTA_HIP(rta::launch_mlp_rows(m->dev, x, nullptr, nullptr, (int)B, Bpad, out, false, (hipStream_t)stream));
  return RTA_OK;
}

static rta_status mlp_loss_grad(rta_mlp* m, const float* x, const float* label, const float* log10e,
                                const int64_t* rows, int64_t n_data, int64_t B, float* loss, hipStream_t st) {
  if (!m) return fail(RTA_E_INVALID_ARG, "null network");
  if (!m->has_params) return fail(RTA_E_INVALID_ARG, "network parameters not set");
  if (B < 1 || B > m->max_batch) return fail(RTA_E_SHAPE, "batch must be in [1, max_batch]");
  if (!x || !label || !log10e) return fail(RTA_E_INVALID_ARG, "null input");
  const int Bpad = (int)((B + 63) & ~63LL);
  RTA_HIP(rta::launch_mlp_rows_gather(m->dev, x, label, log10e, rows, n_data, (int)B, Bpad, nullptr, true, st));
  RTA_HIP(rta::launch_mlp_grad(m->dev, (int)B, Bpad, loss, st));
  m->last_B = B;
  return RTA_OK;
}

static rta_status mlp_adam(rta_mlp* m, hipStream_t st) {
  m->step += 1;
  const double c1 = 1.0 / (1.0 - std::pow((double)m->beta1, (double)m->step));
  const double c2 = 1.0 / (1.0 - std::pow((double)m->beta2, (double)m->step));
  RTA_HIP(rta::launch_mlp_adam(m->dev, true, m->lr, m->beta1, m->beta2, m->eps, (float)c1, (float)c2, st));
  return RTA_OK;
}

rta_status rta_mlp_loss_grad(rta_mlp* m, const float* x, const float* label, const float* log10e, int64_t B,
                             float* grad, float* loss, rta_stream stream) {
  rta_status s = mlp_loss_grad(m, x, label, log10e, nullptr, 0, B, loss, (hipStream_t)stream);
  if (s != RTA_OK) return s;
  RTA_HIP(rta::launch_mlp_grad_sum(m->dev, (hipStream_t)stream));
  if (grad)
    RTA_HIP(hipMemcpyAsync(grad, m->dev.grad, sizeof(float) * rta::kNParams, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
  return RTA_OK;
}

rta_status rta_mlp_train_step(rta_mlp* m, const float* x, const float* label, const float* log10e, int64_t B,
                              float* loss, rta_stream stream) {
  rta_status s = mlp_loss_grad(m, x, label, log10e, nullptr, 0, B, loss, (hipStream_t)stream);
  if (s != RTA_OK) return s;
  return mlp_adam(m, (hipStream_t)stream);
}

rta_status rta_mlp_train_step_rows(rta_mlp* m, const float* x, const float* label, const float* log10e,
                                   int64_t n_data, const int64_t* rows, int64_t B, float* loss, rta_stream stream) {
  if (n_data < 1) return fail(RTA_E_SHAPE, "n_data must be >= 1");
  if (!rows) return fail(RTA_E_INVALID_ARG, "null rows");
  rta_status s = mlp_loss_grad(m, x, label, log10e, rows, n_data, B, loss, (hipStream_t)stream);
  if (s != RTA_OK) return s;
  return mlp_adam(m, (hipStream_t)stream);
}

rta_status rta_mlp_stored(const rta_mlp* m, int32_t which, int64_t B, uint16_t* out, rta_stream stream) {
  if (!m || !out) return fail(RTA_E_INVALID_ARG, "null network or output");
  if (which < 0 || which >= RTA_MLP_STORED_COUNT) return fail(RTA_E_INVALID_ARG, "which must be in [0, 8)");
  if (m->last_B == 0) return fail(RTA_E_INVALID_ARG, "no loss_grad / train_step pass yet");
  if (B != m->last_B) return fail(RTA_E_SHAPE, "B must be the batch size of the last pass");
  const uint16_t* src[RTA_MLP_STORED_COUNT] = {m->dev.H0, m->dev.H1, m->dev.H2, m->dev.H3,
                                               m->dev.G1, m->dev.G2, m->dev.G3, m->dev.G4};
  const size_t rows = (which == 0 || which == 7) ? 16 : 64;  // padded input / output width, hidden width
  const size_t Bpad = (size_t)((B + 63) & ~63LL);
  RTA_HIP(hipMemcpy2DAsync(out, (size_t)B * 2, src[which], Bpad * 2, (size_t)B * 2, rows, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
  return RTA_OK;
}

}  // extern "C"

namespace {
void fill_event_args(const rta_pipeline* pipe, rta::EventArgs& ea) {
  std::memset(&ea, 0, sizeof(ea));
  for (size_t i = 0; i < pipe->cams.size(); ++i) ea.focal[i] = pipe->cams[i]->dev.focal;
  ea.n_types = (int32_t)pipe->cams.size();
  ea.max_width_ratio = pipe->params.max_width_ratio > 0.f ? pipe->params.max_width_ratio : 0.9f;
  ea.max_cond = pipe->params.max_cond > 1.f ? pipe->params.max_cond : 1e4f;
  ea.have_box = pipe->have_box ? 1 : 0;
  ea.have_mlp = pipe->mlp ? 1 : 0;
  if (pipe->mlp) ea.mlp = pipe->mlp->dev;
  if (pipe->have_box) ea.bc = pipe->bc;
}
}  // namespace
