/*
 * rta.h — C ABI of the MI355X low-level reconstruction library (librta.so).
 *
 * The real-time analysis reconstructs every camera event of the DL0 stream
 * built by the Central Event Builder, event by event (paper, Sections 4.1 and
 * 4.2): it calibrates the raw waveforms and produces the per-telescope image
 * parameters from which gamma/hadron separation, energy and direction are
 * derived.  The paper names these products but gives no formulas; the
 * operations below implement the following definitions.
 *
 *   Gain selection   a pixel uses its low-gain trace iff its highest raw
 *                    high-gain sample is >= hg_switch_adc (dual-gain only).
 *   Extraction       W(s) = sum_{k<w} x[s+k] on the selected gain,
 *                    S = W(s*); peak = s* + earliest argmax of x[s*..s*+w-1].
 *                    The window start s* comes from the signal extractor
 *                    (the paper's Section 5 plans several extraction
 *                    algorithms on the GPU; four are provided):
 *                    RTA_EXTRACT_SLIDING: the earliest maximiser of W(s) over
 *                      s in [0, T-w] (the default);
 *                    RTA_EXTRACT_FIXED: s* = the camera's fixed_start for
 *                      every pixel; the gain decision looks only at the
 *                      high-gain samples fixed_start .. fixed_start+w-1, and
 *                      nothing outside the window is read;
 *                    RTA_EXTRACT_GLOBAL_PEAK: s* = the earliest maximiser of
 *                      the camera sum over pixels of the raw high-gain W(s),
 *                      common to every pixel of the event;
 *                    RTA_EXTRACT_NEIGHBOUR_PEAK: per pixel, s* = the earliest
 *                      maximiser of the sum over the pixel's neighbours of
 *                      their raw high-gain W(s) (s* = 0 for a pixel without
 *                      neighbours); the gain decision as for SLIDING.
 *   Calibration      P = nearest-even(256 * ped) (Q8 fixed point),
 *                    D = 256*S - w*P,  q = D / (256 * adc_per_pe)  [p.e.],
 *                    Nt = sum_{k<w} k*(256*x[s*+k] - P),
 *                    t = s* + Nt/D for D > 0, else s* + (w-1)/2  [samples].
 *   Cleaning         thresholds Tx = ceil(256 * adc_per_pe * level) (exact);
 *                    mask_i = (D_i >= Tb_i and a neighbour has D_j >= Tp_j)
 *                          or (D_i >= Tp_i and a neighbour has D_j >= Tb_j),
 *                    every threshold taken at that pixel's selected gain.
 *   Hillas           charge-weighted, centred moments over the mask: size,
 *                    centre of gravity, length = sqrt(l+), width =
 *                    sqrt(l-) with l+ >= l- the eigenvalues of the charge-
 *                    weighted covariance (l- taken as the second moment
 *                    about the major axis), psi in (-pi/2, pi/2],
 *                    skewness / kurtosis of the longitudinal coordinate
 *                    l = (x - cog_x) cos psi + (y - cog_y) sin psi, the
 *                    unweighted least-squares slope / intercept of t over l,
 *                    leakage (charge fraction on pixels with < 6 neighbours),
 *                    number of islands (connected components of the mask).
 *                    Fewer than two mask pixels: the invalid flag is set and
 *                    every float field except size is NaN.
 *   Stereo           point p of the nominal frame (camera metres / focal
 *                    length) minimising sum_i w_i (n_i . (p - cog_i/f_i))^2,
 *                    n_i = (-sin psi_i, cos psi_i), w_i = size (1 - width /
 *                    length); telescopes with invalid Hillas or width/length
 *                    > max_width_ratio are dropped; fewer than two, or a
 *                    normal matrix with condition number >= max_cond, give
 *                    NaN and the invalid flag.
 *
 * Trace layout (one camera event, uint16): [G][T][Npad] — gain, then sample,
 * then pixel, with Npad = round_up(N, 8) (pad pixels are ignored).  One event
 * occupies G*T*Npad elements; its first element must be 16-byte aligned.
 *
 * Conventions.  Pointers named in a stage call are DEVICE pointers owned by
 * the caller unless stated otherwise; the library never frees them and never
 * allocates on their behalf.  Every stage call is asynchronous on the given
 * HIP stream (NULL = the null stream) and never synchronises it; host-side
 * argument checks run before anything is launched and return an error code
 * without launching.  Data errors found inside kernels (a bad descriptor) set
 * bits in the pipeline's device status word and the record's flags; kernels
 * never trap.  Camera handles are immutable after creation and may be
 * shared by threads.  A pipeline's settings change only through
 * rta_set_schedule, rta_pipeline_tune and rta_pipeline_attach_mlp, which must
 * not run concurrently with other calls on that pipeline (rta_pipeline_tune
 * also launches and synchronises its stream); calls that reuse a pipeline's
 * work queue (rta_process_batch, its graphs) must not overlap on different
 * streams.  A graph keeps the schedule and the classifier attachment it was
 * captured with (a network's weights are read from its device memory at
 * every replay).
 */
#ifndef RTA_H
#define RTA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTA_VERSION 1
#define RTA_MAX_PIX 2048      /* largest camera (pixels) */
#define RTA_MAX_SAMP 255      /* largest trace length */
#define RTA_MAX_TYPES 8       /* camera types per pipeline */

/* signal extractors (window placement, see Extraction above) */
#define RTA_EXTRACT_SLIDING 0
#define RTA_EXTRACT_FIXED 1
#define RTA_EXTRACT_GLOBAL_PEAK 2
#define RTA_EXTRACT_NEIGHBOUR_PEAK 3

typedef enum rta_status {
  RTA_OK = 0,
  RTA_E_INVALID_ARG = 1,  /* null handle/pointer, negative count, misalignment */
  RTA_E_SHAPE = 2,        /* unsupported size: N > RTA_MAX_PIX, T > RTA_MAX_SAMP, window not compiled */
  RTA_E_HIP = 3,          /* a HIP runtime call failed (message in rta_last_error) */
  RTA_E_NOMEM = 4,        /* device or host allocation for a handle failed */
  RTA_E_UNSUPPORTED = 5,  /* schedule or option not available */
  RTA_E_UNTUNED = 6       /* the tune cache holds no schedule for this pipeline's key */
} rta_status;

/* record flag bits (rta_hillas_rec.flags) */
#define RTA_FLAG_HILLAS_INVALID 0x1u  /* fewer than two mask pixels */
#define RTA_FLAG_TIME_INVALID 0x2u    /* time gradient undefined (all l equal) */
#define RTA_FLAG_LOW_GAIN 0x4u        /* at least one pixel used its low gain */
#define RTA_FLAG_BAD_DESCRIPTOR 0x8u  /* telescope descriptor rejected in-kernel */
#define RTA_FLAG_MLP_FALLBACK 0x10u   /* box cuts used instead of the network */
/* event flag bits (rta_event_rec.flags) */
#define RTA_EVT_STEREO_INVALID 0x1u
#define RTA_EVT_NO_MLP 0x2u
/* device status word bits (rta_batch_status) */
#define RTA_STATUS_BAD_TYPE 0x1u
#define RTA_STATUS_BAD_OFFSET 0x2u
#define RTA_STATUS_BAD_EVENT 0x4u
#define RTA_STATUS_BAD_PACKET 0x8u

typedef void* rta_stream; /* hipStream_t */

typedef struct rta_camera rta_camera;
typedef struct rta_pipeline rta_pipeline;
typedef struct rta_graph rta_graph;
typedef struct rta_mlp rta_mlp;
typedef struct rta_sam rta_sam;

/* Camera type description.  All pointers are HOST memory, read during
 * rta_camera_create only (copied to device tables). */
typedef struct rta_camera_desc {
  int32_t n_pix;          /* N, 1..RTA_MAX_PIX */
  int32_t n_samp;         /* T, window..RTA_MAX_SAMP */
  int32_t n_gain;         /* 1 or 2 (0 = high, 1 = low gain) */
  int32_t window;         /* w, compiled set: 4 */
  int32_t hg_switch_adc;  /* low gain iff max raw high-gain sample >= this */
  int32_t max_nbr;        /* columns of nbr, <= 6 */
  const float* pix_x;     /* [N] metres */
  const float* pix_y;     /* [N] metres */
  const int32_t* nbr;     /* [N][max_nbr] neighbour pixel indices, -1 padded */
  const float* ped;       /* [G][N] pedestal per sample, ADC */
  const float* adc_per_pe;/* [G][N] ADC counts per photo-electron, > 0 */
  float focal_m;          /* focal length (stereo nominal frame) */
  float t_pic;            /* picture level, p.e. */
  float t_bnd;            /* boundary level, p.e., <= t_pic */
  int32_t fixed_start;    /* first sample of the fixed window, 0..n_samp-window */
} rta_camera_desc;

typedef struct rta_camera_info {
  int32_t n_pix, n_pix_pad, n_samp, n_gain, window, fixed_start;
  int64_t event_elems;    /* uint16 elements per camera event: G*T*Npad */
} rta_camera_info;

/* Per-telescope image record, 64 bytes. */
typedef struct rta_hillas_rec {
  float size, cog_x, cog_y, length, width, psi, skewness, kurtosis;
  float time_gradient, time_intercept, leakage, cog_dist;
  int32_t n_pix, n_islands, n_lowgain;
  uint32_t flags;
} rta_hillas_rec;

/* Per-array-event record, 32 bytes. */
typedef struct rta_event_rec {
  float dir_x, dir_y;     /* nominal frame, radians */
  float cond;             /* condition number of the stereo normal matrix */
  float gammaness;        /* size-weighted mean gamma score (NaN without a network) */
  float log10_energy;     /* size-weighted mean log10(E / TeV) */
  int32_t n_tel, n_used;
  uint32_t flags;
} rta_event_rec;

/* A ragged batch of array events.  Every pointer is DEVICE memory. */
typedef struct rta_batch {
  const uint16_t* traces;       /* trace pool base (16-byte aligned) */
  int64_t traces_len;           /* pool length in uint16 elements */
  const int64_t* evt_tel_off;   /* [n_evt + 1] telescopes of event e: [off[e], off[e+1]) */
  const int32_t* tel_type;      /* [n_tel] index into the pipeline's camera list */
  const int64_t* tel_trace_off; /* [n_tel] element offset of the telescope's trace block (multiple of 8) */
  int64_t n_evt;
  int64_t n_tel;
  uint64_t* evt_done_clock;     /* NULLABLE [n_evt]: with do_stereo, the device clock (see
                                   rta_device_clock_hz) at which each event record was written */
  float* tel_class;             /* NULLABLE [n_tel][2]: with a classifier attached
                                   (rta_pipeline_attach_mlp or rta_pipeline_params.mlp), each telescope is classified in the
                                   reconstruction kernel right after its Hillas parameters: gamma
                                   score and log10(E / TeV) here (NaN without a valid image),
                                   RTA_FLAG_MLP_FALLBACK in its record; the per-event pass then
                                   aggregates these.  Values equal rta_classify's. */
} rta_batch;

typedef struct rta_pipeline_params {
  int32_t do_stereo;        /* 1: per-event stereo + event records */
  int32_t extractor;        /* RTA_EXTRACT_*; extractors other than SLIDING always
                               run one workgroup per telescope (wg_per_cu ignored) */
  float max_width_ratio;    /* stereo: drop images with width/length above (0.9) */
  float max_cond;           /* stereo: invalid at condition number >= this (1e4) */
  const char* tune_cache;   /* NULLABLE path of a schedule tune cache (read at creation, copied):
                               NULL runs the default schedule.  Otherwise the pipeline takes
                               the schedule the cache holds for its tune key; if the file has no
                               such entry (or does not exist), rta_process_batch,
                               rta_process_batch_noalloc and rta_graph_capture return
                               RTA_E_UNTUNED until rta_pipeline_tune or rta_set_schedule has
                               set a schedule, and rta_pipeline_tune records its result in
                               this file. */
  rta_mlp* mlp;              /* NULLABLE: the network classifying each telescope (gamma/hadron
                               score and energy, Section 4.1), attached at creation as by
                               rta_pipeline_attach_mlp(pipe, mlp, boxcut); set with boxcut or
                               not at all (RTA_E_INVALID_ARG otherwise).  Not owned: it must
                               outlive the pipeline or be detached first. */
  const struct rta_boxcut_desc* boxcut;  /* NULLABLE HOST: the box-cut fallback tables (copied) */
} rta_pipeline_params;

/* Launch schedule of the fused kernel (chosen by the autotuner).  A new
 * pipeline starts at {8, 4, 0, 8}, the fastest schedule measured for the
 * mixed 1855/1764/2048-pixel dual-gain workload on MI355X. */
typedef struct rta_schedule {
  int32_t pix_per_lane;     /* 2, 4 or 8 pixels per lane (4-, 8- or 16-byte slice loads) */
  int32_t waves_per_wg;     /* 4 or 8 (256 or 512 threads) */
  int32_t wg_per_cu;        /* 0: one workgroup per telescope (hardware dispatch);
                               1..4: persistent workgroups per compute unit pulling
                               telescopes from a device work queue */
  int32_t chunk;            /* samples per double-buffered load chunk: 8 or 16 */
} rta_schedule;

const char* rta_status_str(rta_status s);
/* Message of the last failing call on this host thread ("" if none). */
const char* rta_last_error(void);
int32_t rta_version(void);
/* Number of compute units of the current device (for schedules). */
rta_status rta_device_cus(int32_t* n_cu);
/* Rate of the device clock that rta_device_stamp and rta_batch.evt_done_clock
 * read (a constant-rate counter, independent of the shader clock), in Hz. */
rta_status rta_device_clock_hz(int64_t* hz);
/* Writes the device clock to *slot (DEVICE uint64) when the stream reaches
 * this point: stamps the completion of earlier work on that stream (for
 * example a host-to-device copy) on the clock of evt_done_clock. */
rta_status rta_device_stamp(uint64_t* slot, rta_stream stream);

/* Create / destroy a camera type.  Quantises pedestals to Q8 and builds the
 * integer cleaning thresholds and neighbour tables on the current device.
 * The camera's device memory also holds the health monitor's scratch:
 * 512 partial blocks of 3 * n_gain * n_pix_pad 64-bit sums (50 MB for a
 * 2048-pixel dual-gain type). */
rta_status rta_camera_create(const rta_camera_desc* desc, rta_camera** out);
rta_status rta_camera_destroy(rta_camera* cam);
rta_status rta_camera_get_info(const rta_camera* cam, rta_camera_info* info);

/* Calibration + extraction of n_evt camera events of one type with the
 * sliding-window extractor.  traces: [n_evt][G][T][Npad].  Outputs
 * [n_evt][N], each NULLABLE: S, D (int32), sstar, peak, gain (uint8),
 * q (p.e.), t (samples) as float. */
rta_status rta_calibrate(const rta_camera* cam, const uint16_t* traces, int64_t n_evt, int32_t* S, int32_t* D,
                         uint8_t* sstar, uint8_t* peak, uint8_t* gain, float* q, float* t, rta_stream stream);
/* The same with any extractor (RTA_EXTRACT_*; RTA_E_INVALID_ARG otherwise). */
rta_status rta_calibrate_ex(const rta_camera* cam, int32_t extractor, const uint16_t* traces, int64_t n_evt,
                            int32_t* S, int32_t* D, uint8_t* sstar, uint8_t* peak, uint8_t* gain, float* q,
                            float* t, rta_stream stream);

/* Cleaning levels of one rta_clean call, photo-electrons. */
typedef struct rta_clean_params {
  float t_pic;              /* picture level */
  float t_bnd;              /* boundary level, <= t_pic */
} rta_clean_params;

/* Two-level tailcut (image cleaning, Section 4.1) of n_evt events: a pixel
 * stays if it is at or above the boundary level with a neighbour at or above
 * the picture level, or at or above the picture level with a neighbour at or
 * above the boundary level, on the integer thresholds ceil(256 a T) of D
 * (Q8).  levels: NULLABLE host struct; NULL takes the camera's levels (the
 * ones the fused path uses); otherwise finite with t_bnd <= t_pic and
 * |256 a T| <= 2e9 for every pixel's a, else RTA_E_INVALID_ARG.  D, gain:
 * [n_evt][N] device (gain NULLABLE = all high gain).  mask: [n_evt][N] 0/1. */
rta_status rta_clean(const rta_camera* cam, const rta_clean_params* levels, const int32_t* D, const uint8_t* gain,
                     int64_t n_evt, uint8_t* mask, rta_stream stream);

/* Hillas parameters (Section 4.1) of n_evt events from calibrated charges
 * q_pe (p.e., as rta_calibrate writes them), peak times t (samples) and the
 * cleaning mask, all [n_evt][N] device.  gain: NULLABLE [n_evt][N]; when
 * given, the record's n_lowgain and RTA_FLAG_LOW_GAIN count the low-gain
 * pixels of the image (as the fused path does); NULL counts none.  out:
 * [n_evt] records.  With q_pe and t from rta_calibrate and the mask from
 * rta_clean, every field but the time regression equals the fused path's
 * record bit for bit (the fused path keeps peak times in FP64, t is FP32). */
rta_status rta_hillas(const rta_camera* cam, const float* q_pe, const float* t, const uint8_t* mask,
                      const uint8_t* gain, int64_t n_evt, rta_hillas_rec* out, rta_stream stream);
/* The same from the integer calibration output: D (Q8, [n_evt][N] device)
 * and its gain (NULLABLE = all high gain, then also no low-gain count); the
 * charge D / (256 a) is formed in the kernel as rta_calibrate forms q_pe, so
 * the records equal rta_hillas's on rta_calibrate's q_pe and gain. */
rta_status rta_hillas_q8(const rta_camera* cam, const int32_t* D, const float* t, const uint8_t* mask,
                         const uint8_t* gain, int64_t n_evt, rta_hillas_rec* out, rta_stream stream);

/* A pipeline over 1..RTA_MAX_TYPES camera types (the handles must outlive it). */
rta_status rta_pipeline_create(rta_camera* const* cams, int32_t n_types, const rta_pipeline_params* params,
                               rta_pipeline** out);
rta_status rta_pipeline_destroy(rta_pipeline* pipe);
rta_status rta_set_schedule(rta_pipeline* pipe, const rta_schedule* s);
rta_status rta_get_schedule(const rta_pipeline* pipe, rta_schedule* s);
/* All schedules compiled into the library; *n receives the count. */
rta_status rta_list_schedules(rta_schedule* out, int32_t cap, int32_t* n);

/* The fused path: one kernel runs calibration -> cleaning -> Hillas for
 * every telescope of the batch (one workgroup per telescope, or persistent
 * workgroups on a dynamic work queue, per the schedule), then (if do_stereo)
 * one pass per array event computes stereo, network scores and the event
 * record.  tel_out: [n_tel]; evt_out: [n_evt] (NULLABLE when
 * do_stereo == 0). */
rta_status rta_process_batch(rta_pipeline* pipe, const rta_batch* batch, rta_hillas_rec* tel_out,
                             rta_event_rec* evt_out, rta_stream stream);

/* Allocation-free form of rta_process_batch, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same kernels, arguments, checks and
 * records as rta_process_batch with the pipeline pipe (its cameras, params,
 * schedule and attached network); the work-queue counter and the status word
 * live in a static device array of RTA_NOALLOC_SCRATCH_BYTES bytes, one per
 * GPU, held until the process ends, instead of the pipeline's device memory.
 * The call allocates nothing (no hipMalloc / hipFree, no allocating library
 * routine); its first call on a device looks up that device's copy of the
 * array.  The scratch need is fixed (a 64-bit counter and a 32-bit word,
 * within the 256 bytes) and does not grow with the batch, so batches are
 * limited exactly as for rta_process_batch.
 * status_out: NULLABLE device uint32; receives, on the stream, the
 * RTA_STATUS_* bits of this call's batch alone (the scratch status word is
 * cleared at the start of the call; the pipeline's own status word is not
 * touched).  The pipeline's device must be the current device, else
 * RTA_E_INVALID_ARG.  Every call on one GPU shares that GPU's scratch: calls
 * that overlap on one GPU (different streams or threads) race and must not be
 * issued. */
#define RTA_NOALLOC_SCRATCH_BYTES 256
rta_status rta_process_batch_noalloc(const rta_pipeline* pipe, const rta_batch* batch, rta_hillas_rec* tel_out,
                                     rta_event_rec* evt_out, uint32_t* status_out, rta_stream stream);

/* Schedule tuning.  A launch-configuration search, not a step of the
 * reconstruction: records and statuses are the same under every schedule.
 *
 * Tune key of a pipeline: "<arch>|e<extractor>w<window>|<N>x<T>x<G>;..." over
 * its camera types in order, arch being the device's gfx name ("gfx950").
 * key: host buffer of cap bytes (RTA_TUNE_KEY_MAX suffices); RTA_E_INVALID_ARG
 * if it does not fit. */
#define RTA_TUNE_KEY_MAX 512
rta_status rta_pipeline_tune_key(const rta_pipeline* pipe, char* key, int32_t cap);

/* Times candidate schedules of the fused path on one batch and applies the
 * fastest.  Each candidate runs one untimed rta_process_batch, then reps
 * (1..100) timed ones bracketed by HIP events on stream; its time is the
 * median.  cands: NULLABLE host array of n_cands schedules (all must be
 * compiled, else RTA_E_UNSUPPORTED before any launch); NULL times every
 * compiled schedule (rta_list_schedules) and ignores n_cands.  ms: NULLABLE
 * host array, one median per candidate in milliseconds.  best: NULLABLE,
 * receives the chosen schedule.  Batch, outputs and validation as for
 * rta_process_batch (the outputs hold the last run's records afterwards).
 * Synchronises the stream.  If the pipeline was created with a tune cache, the
 * result is stored there under the pipeline's key (replacing an older entry;
 * an unwritable file gives RTA_E_INVALID_ARG after the schedule is applied).
 * On a failed launch the previous schedule is kept. */
rta_status rta_pipeline_tune(rta_pipeline* pipe, const rta_batch* batch, rta_hillas_rec* tel_out,
                             rta_event_rec* evt_out, const rta_schedule* cands, int32_t n_cands, int32_t reps,
                             float* ms, rta_schedule* best, rta_stream stream);

/* The tune cache file: UTF-8 text, one entry per line,
 * "<key>\t<pix_per_lane> <waves_per_wg> <wg_per_cu> <chunk>\t<ms>"; lines
 * starting with '#' and lines that do not parse are ignored.  Host-only calls
 * (no GPU use).  Lookup: RTA_E_UNTUNED when the file is missing or holds no
 * parseable entry for key, or when the entry's schedule is not compiled into
 * this library; ms NULLABLE.  Store: replaces the key's entry (or appends one)
 * and rewrites the file through a temporary file renamed over it, so readers
 * see the old or the new file; keys may not hold tabs or line breaks. */
rta_status rta_tune_cache_lookup(const char* path, const char* key, rta_schedule* s, float* ms);
rta_status rta_tune_cache_store(const char* path, const char* key, const rta_schedule* s, float ms);

/* Stereo per array event from existing telescope records, using the
 * pipeline's focal lengths and cuts.  evt_tel_off [n_evt+1] (values in
 * [0, n_tel]), tel_type [n_tel], tel [n_tel], evt_out [n_evt]. */
rta_status rta_stereo(rta_pipeline* pipe, const int64_t* evt_tel_off, const int32_t* tel_type, int64_t n_evt,
                      int64_t n_tel, const rta_hillas_rec* tel, rta_event_rec* evt_out, rta_stream stream);

/* Synchronises the pipeline's status read: copies the device status word
 * (RTA_STATUS_* bits accumulated since the last call) and clears it. */
rta_status rta_batch_status(rta_pipeline* pipe, uint32_t* status);

/* Capture rta_process_batch(pipe, batch, ...) with these exact pointers and
 * sizes into a HIP graph (captured on a library-owned stream); replay it with
 * rta_graph_launch on any stream.  The batch's device arrays may be rewritten
 * between replays; their sizes may not. */
rta_status rta_graph_capture(rta_pipeline* pipe, const rta_batch* batch, rta_hillas_rec* tel_out,
                             rta_event_rec* evt_out, rta_graph** out);
rta_status rta_graph_launch(rta_graph* g, rta_stream stream);
rta_status rta_graph_destroy(rta_graph* g);

/* ------------------------------------------------------------------------
 * DL0 telemetry packets: the byte stream of camera events between the event
 * builder and the analysis, formatted in the manner of space telemetry
 * source packets (paper, Section 5).  One packet per camera event, every
 * multi-byte field big-endian:
 *    0  u16  packet id: version 0 (3 bits) | type 0 (1 bit) | secondary
 *            header flag 1 (1 bit) | APID = telescope id (11 bits)
 *    2  u16  sequence control: flags 0b11 (2 bits) | sequence count (14 bits)
 *    4  u32  packet data length = total packet length - 9
 *    8  u8   0x10    9  u8 service 210    10  u8 subtype 1
 *   11  u8   camera type (index into the pipeline's camera list)
 *   12  u32  coarse time    16  u16 fine time
 *   18  u16  n_pix    20  u16 n_samp    22  u8 n_gain    23  u8 spare (0)
 *   24  u64  event number
 *   32  u16  samples [G][T][N] (no padding)
 *  end  u16  CRC-16 of every byte before it: polynomial x^16+x^12+x^5+1,
 *            register 0xFFFF, most significant bit first, no final xor.
 * ------------------------------------------------------------------------ */
#define RTA_PACKET_PAD 32          /* readable bytes required after a packet stream */
#define RTA_PKT_HEADER_BAD 0x1u  /* fixed fields, flags or length inconsistent */
#define RTA_PKT_TYPE_BAD 0x2u    /* camera type unknown / dimensions differ / no pool slot */
#define RTA_PKT_CRC_BAD 0x4u     /* CRC mismatch */

/* Per-packet record written by rta_decode_packets, 32 bytes. */
typedef struct rta_packet_rec {
  uint64_t event_number;
  uint32_t coarse_time;
  uint16_t fine_time, apid, seq_count, cam_type;
  uint32_t flags;                     /* RTA_PKT_* */
  uint16_t crc_stored, crc_computed;  /* valid when the header and type were good */
  uint32_t pad_;
} rta_packet_rec;

/* Framing on the host (all pointers HOST memory; nothing is launched):
 * walks the packet headers of bytes[0, n_bytes) from offset 0.  For each
 * whole packet (at most cap): pkt_off = its byte offset; tel_type = its
 * camera type if that is < n_types and the header's n_pix / n_samp / n_gain
 * equal types[t]'s, else -1; tel_trace_off = the element offset of its slot
 * in the decoded pool (slots of G*T*Npad elements in packet order; 0 and no
 * slot for type -1).  Outputs the packet count, the pool size in elements
 * and the bytes consumed (the start of a trailing partial packet, which
 * belongs to the next chunk).  RTA_E_SHAPE if a data length implies a
 * packet shorter than 34 bytes (framing lost; *consumed = its offset). */
rta_status rta_frame_packets(const rta_camera_info* types, int32_t n_types, const uint8_t* bytes, int64_t n_bytes,
                             int64_t cap, int64_t* pkt_off, int32_t* tel_type, int64_t* tel_trace_off,
                             int64_t* n_pkt, int64_t* pool_elems, int64_t* consumed);

/* Decode on the device (all pointers DEVICE memory): one workgroup per
 * packet checks the header, the camera type against tel_type[p] and the
 * pipeline's camera dimensions, and the CRC (computed in parallel, each
 * lane folding its 16-byte column pieces by the linearity of the CRC over
 * GF(2)), and writes the samples little-endian into pool[tel_trace_off[p]
 * ...] as [G][T][Npad] with zero pad columns.  A packet failing any check
 * gets tel_type[p] = -1 (in place: the fused batch then flags it as a bad
 * descriptor), its record's flags and RTA_STATUS_BAD_PACKET in the status
 * word; a CRC failure is known only after its slot was written.  A packet
 * offset outside [0, n_bytes - 34] reads nothing and is flagged
 * RTA_PKT_HEADER_BAD.
 * bytes: 16-byte aligned, and the RTA_PACKET_PAD bytes after bytes[n_bytes]
 * must be readable (their content is ignored).  rec: [n_pkt], NULLABLE. */
rta_status rta_decode_packets(rta_pipeline* pipe, const uint8_t* bytes, int64_t n_bytes, const int64_t* pkt_off,
                              int32_t* tel_type, const int64_t* tel_trace_off, int64_t n_pkt, uint16_t* pool,
                              int64_t pool_elems, rta_packet_rec* rec, rta_stream stream);

/* ------------------------------------------------------------------------
 * Gamma/hadron + energy network (the separation and energy steps of the
 * reconstruction products, Section 4.1): 10 per-telescope features ->
 * 64 -> 64 -> 64 (ReLU) -> [gamma logit, log10(E/TeV)], bfloat16 operands
 * with FP32 accumulation on the matrix cores, FP32 master weights + Adam.
 * Features, in order: log10(size), length, width, cog_dist, psi, skewness,
 * kurtosis, time_gradient, leakage, n_islands; standardised inside the
 * kernels with the mean / std given to rta_mlp_set_params.
 * Loss: mean over the batch of BCE(logit, label) + label * (log10 E - y)^2.
 * Parameters are packed as W1 [10][64], b1 [64], W2 [64][64], b2, W3 [64][64],
 * b3, W4 [64][2], b4 [2] (W[in][out]), 9154 floats.
 * ---------------------------------------------------------------------- */
#define RTA_MLP_N_PARAMS 9154
#define RTA_MLP_N_FEATURES 10

typedef struct rta_mlp_desc {
  int32_t max_batch;      /* largest training batch (scratch is sized for it) */
  float lr, beta1, beta2, eps;  /* Adam */
} rta_mlp_desc;

rta_status rta_mlp_create(const rta_mlp_desc* desc, rta_mlp** out);
rta_status rta_mlp_destroy(rta_mlp* m);
/* HOST arrays: params [RTA_MLP_N_PARAMS], feat_mean / feat_std [10] (std > 0).
 * Uploads the FP32 masters, rebuilds the bf16 copies, resets Adam.
 * Synchronous. */
rta_status rta_mlp_set_params(rta_mlp* m, const float* params, const float* feat_mean, const float* feat_std);
/* Copies the FP32 master parameters to HOST params [RTA_MLP_N_PARAMS]; synchronous. */
rta_status rta_mlp_get_params(rta_mlp* m, float* params);
/* Inference: x [B][10] raw features (device) -> out [B][2] (device). */
rta_status rta_mlp_forward(rta_mlp* m, const float* x, int64_t B, float* out, rta_stream stream);
/* Loss and gradient of one batch (B <= max_batch): label [B] (1 gamma, 0
 * hadron), log10e [B] (used for gammas).  grad: device [RTA_MLP_N_PARAMS]
 * (NULLABLE), loss: device scalar (NULLABLE).  Weights are not changed.
 * The batch sums run in a fixed order, so equal inputs give bit-equal
 * results.  loss_grad and train_step use the network's per-batch scratch
 * and train_step rewrites its weights: issue the calls on one network from
 * one stream (calls that overlap on the device race). */
rta_status rta_mlp_loss_grad(rta_mlp* m, const float* x, const float* label, const float* log10e, int64_t B,
                             float* grad, float* loss, rta_stream stream);
/* One training step: loss_grad then an Adam update of the masters and the
 * bf16 copies.  loss: device scalar (NULLABLE). */
rta_status rta_mlp_train_step(rta_mlp* m, const float* x, const float* label, const float* log10e, int64_t B,
                              float* loss, rta_stream stream);
/* The same step on a batch drawn from data arrays: x [n_data][10], label
 * [n_data], log10e [n_data] and rows [B] (all DEVICE); batch row b is data
 * row rows[b] (values outside [0, n_data) are clamped into it), gathered
 * inside the kernel.  Equal to rta_mlp_train_step on the gathered arrays. */
rta_status rta_mlp_train_step_rows(rta_mlp* m, const float* x, const float* label, const float* log10e,
                                   int64_t n_data, const int64_t* rows, int64_t B, float* loss, rta_stream stream);

/* Inspection of the last loss_grad / train_step(_rows) pass of this network:
 * copies the bfloat16 values that pass stored for the weight-gradient
 * contraction.  which = 0: the standardised input (16 rows; rows 10..15 are
 * zero); 1..3: the hidden activations h1..h3 (64 rows); 4..6: the gradient
 * signals at the pre-activations of layers 1..3 (64 rows, the ReLU mask
 * applied); 7: the gradient at the two outputs (16 rows; rows 2..15 zero).
 * out: DEVICE uint16 (bfloat16 bits) [rows][B], feature-major, B = that
 * pass's batch size (else RTA_E_SHAPE; RTA_E_INVALID_ARG before any pass).
 * Asynchronous on the stream; read it before the network's next pass. */
#define RTA_MLP_STORED_COUNT 8
rta_status rta_mlp_stored(const rta_mlp* m, int32_t which, int64_t B, uint16_t* out, rta_stream stream);

/* ------------------------------------------------------------------------
 * Classification with fallback.  Plain scaled-width / scaled-length box cuts
 * serve as the baseline and as the fallback when a telescope's features are
 * non-finite or outside the range the network was trained on:
 *   bin b = clamp(floor((log10 size - lgs_lo) / (lgs_hi - lgs_lo) * n_bins))
 *   SW = (width - w_mean[b]) / w_std[b],  SL = (length - l_mean[b]) / l_std[b]
 *   gamma iff SW < cut_w and SL < cut_l;  log10 E = e_a + e_b log10 size.
 * With the network: score = sigmoid(logit), gamma iff score > mlp_cut.
 * The tables are prepared from training images by the host (see the Python
 * package); all per-telescope decisions run in the kernels.
 * ---------------------------------------------------------------------- */
#define RTA_BOXCUT_MAX_BINS 32

typedef struct rta_boxcut_desc {
  int32_t n_bins;                 /* 1..RTA_BOXCUT_MAX_BINS */
  float lgs_lo, lgs_hi;           /* log10(size) range of the bins */
  float w_mean[RTA_BOXCUT_MAX_BINS], w_std[RTA_BOXCUT_MAX_BINS];
  float l_mean[RTA_BOXCUT_MAX_BINS], l_std[RTA_BOXCUT_MAX_BINS];
  float cut_w, cut_l;
  float e_a, e_b;
  float feat_lo[RTA_MLP_N_FEATURES], feat_hi[RTA_MLP_N_FEATURES]; /* trained range */
  float mlp_cut;                  /* score threshold of the network */
} rta_boxcut_desc;

/* Network inputs of n Hillas records (device): x [n][10] (device). */
rta_status rta_features(const rta_hillas_rec* rec, int64_t n, float* x, rta_stream stream);

/* Per-telescope classification of n records (device) -> out [n][4] (device):
 * gamma score, log10 E, gamma decision (0/1), fallback used (0/1).  m NULLABLE
 * (box cuts only); bc is HOST memory, read during the call. */
rta_status rta_classify(rta_mlp* m, const rta_boxcut_desc* bc, const rta_hillas_rec* rec, int64_t n, float* out,
                        rta_stream stream);

/* Attach (m != NULL) or detach the network and box cuts to a pipeline.  Every
 * telescope is then classified: in the reconstruction kernel right after its
 * Hillas parameters when the batch gives rta_batch.tel_class, otherwise (with
 * do_stereo) in the per-event pass; RTA_FLAG_MLP_FALLBACK marks records that
 * used the box cuts.  With do_stereo the event record gets the size-weighted
 * mean score and log10 E.  The network must outlive the pipeline or be
 * detached first.  bc: HOST memory. */
rta_status rta_pipeline_attach_mlp(rta_pipeline* pipe, rta_mlp* m, const rta_boxcut_desc* bc);

/* ------------------------------------------------------------------------
 * Real-time health monitor: a quality check of the acquired data whose
 * verdict lets the alert monitor hold back on bad data (paper, Section 4.2).
 * Over n_evt camera events of one type, per gain g and pixel i:
 *   n = n_evt * T samples, s1 = sum x, s2 = sum x^2, n_sat = samples >= the
 *   saturation level (the high-gain switch level for the high gain of a
 *   dual-gain camera, 65535 otherwise); mean = s1 / n, rms = sqrt(max(s2 / n
 *   - mean^2, 0)) in FP64 without contraction; per gain the lower median of
 *   the pixels' rms (element (N-1)/2 of the sorted values); flags
 *   RTA_HEALTH_DEAD rms < rms_dead, RTA_HEALTH_NOISY rms > noisy_factor *
 *   median, RTA_HEALTH_PED_SHIFT |mean - P/256| > ped_tol (P the Q8
 *   pedestal), RTA_HEALTH_SATURATING n_sat > sat_frac * n; verdict 1 when
 *   the pixels with any flag in any gain exceed bad_frac_max * N.
 * ------------------------------------------------------------------------ */
#define RTA_HEALTH_DEAD 0x1u
#define RTA_HEALTH_NOISY 0x2u
#define RTA_HEALTH_PED_SHIFT 0x4u
#define RTA_HEALTH_SATURATING 0x8u

typedef struct rta_health_params {
  float rms_dead, noisy_factor, ped_tol, sat_frac, bad_frac_max;
  int32_t pad_;
} rta_health_params;

/* Per pixel and gain, 64 bytes. */
typedef struct rta_pixel_health {
  uint64_t n, s1, s2, n_sat;
  double mean, rms;
  uint32_t flags, pad_;
  uint64_t reserved_;
} rta_pixel_health;

typedef struct rta_camera_health {
  double median_rms[2];  /* per gain (index 1 unused for single gain) */
  int32_t n_bad;         /* pixels with any flag */
  int32_t verdict;       /* 1: data quality insufficient */
} rta_camera_health;

/* Health statistics of n_evt events of one type: traces [n_evt][G][T][Npad]
 * (DEVICE), pix [G][N] and out (DEVICE).  Uses accumulators owned by the
 * camera: calls on one camera must not overlap. */
rta_status rta_health(rta_camera* cam, const uint16_t* traces, int64_t n_evt, const rta_health_params* params,
                      rta_pixel_health* pix, rta_camera_health* out, rta_stream stream);

/* ------------------------------------------------------------------------
 * Science alert monitor (SAM): search of the event list for transients on
 * several integration timescales, inside a source region and anywhere in the
 * field of view (paper, Section 2 requirement (ii) and Section 4.2).
 *   selection    array events with a valid stereo direction and gammaness
 *                >= gamma_cut
 *   binning      time bin b = floor((t - t0) / bin_s) in [0, n_bins); sky
 *                cell ix = floor(dir_x / cell + grid / 2), iy likewise, in
 *                [0, grid) (nominal frame, radians; evaluated in FP64)
 *   counts       C[b][iy][ix] = selected events
 *   window       for w bins ending at bin e: W = sum of C over e-w < b <= e
 *   on / off     per cell: N_on = sum of W over the cells at squared cell
 *                distance <= r_on^2, N_off over r_in^2 < d^2 <= r_out^2,
 *                both inside the grid; alpha = on cells / off cells
 *   significance Li & Ma (1983) eq. 17 with the sign of N_on - alpha N_off,
 *                0 when the excess is exactly zero (decided in integers),
 *                when N_on + N_off = 0 or without off cells; FP64
 *   alert        significance >= sigma_alert
 * ------------------------------------------------------------------------ */
#define RTA_SAM_MAX_GRID 256
#define RTA_SAM_MAX_SCALES 8
#define RTA_SAM_MAX_REACH 16   /* r_out in cells */

typedef struct rta_sam_params {
  int32_t grid;          /* cells per side, 1..RTA_SAM_MAX_GRID */
  int32_t n_bins;        /* time bins held, >= 1 (counts: n_bins * grid^2 int32) */
  double t0;             /* start of bin 0, s */
  double bin_s;          /* bin width, s, > 0 */
  float cell;            /* cell size, radians, > 0 */
  float r_on, r_in, r_out;  /* radii in cells: 0 <= r_on < r_in < r_out <= RTA_SAM_MAX_REACH */
  float gamma_cut;       /* minimum gammaness */
  float sigma_alert;     /* alert threshold */
  int32_t n_scales;      /* 1..RTA_SAM_MAX_SCALES */
  int32_t scales[RTA_SAM_MAX_SCALES];  /* window lengths in bins, 1..n_bins */
} rta_sam_params;

/* One alert, 32 bytes. */
typedef struct rta_sam_alert {
  int32_t scale;         /* index into scales */
  int32_t ix, iy;        /* cell */
  int32_t n_on;
  double significance;
  int32_t n_off;
  int32_t pad_;
} rta_sam_alert;

/* Create / destroy a monitor on the current device (allocates the counts
 * and window maps; counts start at zero). */
rta_status rta_sam_create(const rta_sam_params* params, rta_sam** out);
rta_status rta_sam_destroy(rta_sam* sam);
/* Zero the counts (a fill kernel, so it may be captured in a graph). */
rta_status rta_sam_clear(rta_sam* sam, rta_stream stream);
/* Add n events to the counts: evt [n] records (DEVICE), t [n] arrival
 * times in s (DEVICE, FP64).  Events outside the bins or the grid are
 * ignored.  Order-independent (integer atomics). */
rta_status rta_sam_fill(rta_sam* sam, const rta_event_rec* evt, const double* t, int64_t n, rta_stream stream);
/* Search the windows ending at bin end_bin (0 <= end_bin < n_bins) for every
 * timescale.  significance [n_scales][grid][grid] FP64, n_on / n_off
 * [n_scales][grid][grid] int32 (each NULLABLE, DEVICE); alerts [max_alerts]
 * (DEVICE) in any order, n_alerts (DEVICE int32) the number found (may exceed
 * max_alerts; only max_alerts are written). */
rta_status rta_sam_search(rta_sam* sam, int32_t end_bin, double* significance, int32_t* n_on, int32_t* n_off,
                          rta_sam_alert* alerts, int32_t max_alerts, int32_t* n_alerts, rta_stream stream);
/* Copy the counts [n_bins][grid][grid] int32 into dst (DEVICE, caller-owned),
 * asynchronously on stream. */
rta_status rta_sam_counts(const rta_sam* sam, int32_t* dst, rta_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* RTA_H */
