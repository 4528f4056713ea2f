/*
 * dl0sim — seeded synthetic DL0 input generator.
 *
 * This module stands in for the Central Event Builder simulator fed by
 * simulated data (Section 5 of the paper): it produces camera geometries,
 * dual-gain uint16 waveform traces of Cherenkov images, ragged array events
 * and charge-domain images.  It holds none of the reconstruction arithmetic
 * (no window sums, calibration, cleaning or moments); both the HIP library and
 * the CPU oracle consume its outputs as plain inputs.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), keyed by the
 * seed and countered by (event, pixel, block, stream), so any event range can
 * be generated in any order or thread split and gives identical bytes.
 *
 * Trace layout written by dl0sim_render_traces (one camera event):
 *   uint16 [G][T][Npad]  — gain-major, then sample (slice), then pixel; pixels
 *   Npad = round_up(N, 8); pad pixels are written as 0.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DL0_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Philox4x32-10                                                        */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t v[4]; } ph_ctr;

static inline void ph_mulhilo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

static ph_ctr philox4x32_10(ph_ctr c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0, lo0, hi1, lo1;
    ph_mulhilo(M0, c.v[0], &hi0, &lo0);
    ph_mulhilo(M1, c.v[2], &hi1, &lo1);
    ph_ctr n;
    n.v[0] = hi1 ^ c.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ c.v[3] ^ k1;
    n.v[3] = lo0;
    c = n;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

/* A stream of uint32 draws for one (seed, event, pixel, stream) tuple. */
typedef struct {
  uint32_t k0, k1;
  uint32_t c0, c1, c2;  /* event lo, event hi | stream<<24, pixel */
  uint32_t block;
  uint32_t buf[4];
  int pos;
} ph_stream;

static void ph_init(ph_stream* s, uint64_t seed, uint64_t event, uint32_t pixel, uint32_t stream) {
  s->k0 = (uint32_t)seed;
  s->k1 = (uint32_t)(seed >> 32);
  s->c0 = (uint32_t)event;
  s->c1 = ((uint32_t)(event >> 32) & 0x00FFFFFFu) | (stream << 24);
  s->c2 = pixel;
  s->block = 0;
  s->pos = 4;
}

static inline uint32_t ph_next(ph_stream* s) {
  if (s->pos == 4) {
    ph_ctr c = {{s->c0, s->c1, s->c2, s->block++}};
    ph_ctr r = philox4x32_10(c, s->k0, s->k1);
    memcpy(s->buf, r.v, sizeof(s->buf));
    s->pos = 0;
  }
  return s->buf[s->pos++];
}

/* uniform in the open interval (0, 1) */
static inline double ph_uniform(ph_stream* s) { return ((double)ph_next(s) + 0.5) * (1.0 / 4294967296.0); }

/* standard normal by the Box–Muller transform (one of the pair is used) */
static inline double ph_normal(ph_stream* s) {
  double u1 = ph_uniform(s), u2 = ph_uniform(s);
  return sqrt(-2.0 * log(u1)) * cos(2.0 * DL0_PI * u2);
}

/* Box–Muller pair */
static inline void ph_normal2(ph_stream* s, double* z0, double* z1) {
  double u1 = ph_uniform(s), u2 = ph_uniform(s);
  double r = sqrt(-2.0 * log(u1));
  *z0 = r * cos(2.0 * DL0_PI * u2);
  *z1 = r * sin(2.0 * DL0_PI * u2);
}

/* Poisson draw: inversion for small means, rounded normal approximation
 * above 40 (a generator approximation; the reconstruction never assumes it). */
static int64_t ph_poisson(ph_stream* s, double lam) {
  if (!(lam > 0.0)) return 0;
  if (lam > 40.0) {
    double k = nearbyint(lam + sqrt(lam) * ph_normal(s));
    return k < 0 ? 0 : (int64_t)k;
  }
  double u = ph_uniform(s);
  double p = exp(-lam), F = p;
  int64_t k = 0;
  while (u > F && k < 1000) {
    ++k;
    p *= lam / (double)k;
    F += p;
  }
  return k;
}

/* ------------------------------------------------------------------ */
/* Camera geometry: hexagonal lattice, the N lattice points closest to  */
/* the origin, ordered by (norm, polar angle in [0, 2pi), a).           */
/* ------------------------------------------------------------------ */
typedef struct { int64_t n2; double ang; int a, b; } hexpt;

static int hexpt_cmp(const void* pa, const void* pb) {
  const hexpt* p = (const hexpt*)pa;
  const hexpt* q = (const hexpt*)pb;
  if (p->n2 != q->n2) return p->n2 < q->n2 ? -1 : 1;
  if (p->ang != q->ang) return p->ang < q->ang ? -1 : 1;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  return 0;
}

/* Lattice neighbour directions in (a, b). */
static const int HEX_DA[6] = {1, 0, -1, -1, 0, 1};
static const int HEX_DB[6] = {0, 1, 1, 0, -1, -1};

/*
 * x, y: [n_pix] metres.  nbr: [n_pix][6] lattice neighbours (-1 where the
 * neighbour is not part of the camera).  ab: optional [n_pix][2] lattice
 * coordinates.  Returns 0 on success.
 */
int dl0sim_camera_geometry(int n_pix, double pitch, float* x, float* y, int32_t* nbr, int32_t* ab) {
  if (n_pix <= 0) return -1;
  int R = 1;
  while (1 + 3 * R * (R + 1) < 2 * n_pix + 64) ++R;
  R += 2;
  int side = 2 * R + 1;
  hexpt* pts = (hexpt*)malloc(sizeof(hexpt) * (size_t)side * side);
  if (!pts) return -2;
  int m = 0;
  for (int a = -R; a <= R; ++a)
    for (int b = -R; b <= R; ++b) {
      int64_t n2 = (int64_t)a * a + (int64_t)a * b + (int64_t)b * b;
      if (n2 > (int64_t)R * R) continue;
      double px = a + 0.5 * b, py = b * (sqrt(3.0) / 2.0);
      double ang = atan2(py, px);
      if (ang < 0) ang += 2.0 * DL0_PI;
      if (n2 == 0) ang = 0.0;
      pts[m].n2 = n2;
      pts[m].ang = ang;
      pts[m].a = a;
      pts[m].b = b;
      ++m;
    }
  if (m < n_pix) { free(pts); return -3; }
  qsort(pts, (size_t)m, sizeof(hexpt), hexpt_cmp);
  /* index lookup over the bounding box */
  int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)side * side);
  if (!idx) { free(pts); return -2; }
  for (int i = 0; i < side * side; ++i) idx[i] = -1;
  for (int i = 0; i < n_pix; ++i) idx[(pts[i].a + R) * side + (pts[i].b + R)] = i;
  for (int i = 0; i < n_pix; ++i) {
    int a = pts[i].a, b = pts[i].b;
    x[i] = (float)(pitch * (a + 0.5 * b));
    y[i] = (float)(pitch * b * (sqrt(3.0) / 2.0));
    if (ab) { ab[2 * i] = a; ab[2 * i + 1] = b; }
    for (int d = 0; d < 6; ++d) {
      int na = a + HEX_DA[d], nb = b + HEX_DB[d];
      int32_t j = -1;
      if (na >= -R && na <= R && nb >= -R && nb <= R) j = idx[(na + R) * side + (nb + R)];
      nbr[6 * i + d] = j;
    }
  }
  free(idx);
  free(pts);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Shower (image) parameters                                            */
/* ------------------------------------------------------------------ */
#define DL0_MAX_BLOB 4

typedef struct dl0sim_shower {
  int32_t n_blob;
  int32_t kind;          /* 0 plain ellipse, 1 gamma, 2 hadron */
  float energy_tev;      /* gammas/hadrons only, else 0 */
  float src_x, src_y;    /* source image in camera metres (array events), else NaN */
  float pad_[3];
  float size[DL0_MAX_BLOB];
  float cog_x[DL0_MAX_BLOB];
  float cog_y[DL0_MAX_BLOB];
  float width[DL0_MAX_BLOB];
  float length[DL0_MAX_BLOB];
  float psi[DL0_MAX_BLOB];
  float t0[DL0_MAX_BLOB];
  float tgrad[DL0_MAX_BLOB];
} dl0sim_shower;

typedef struct dl0sim_draw_cfg {
  double size_min, size_max;       /* log-uniform p.e. */
  double cog_rmax;                 /* m */
  double width_min, width_max;     /* m */
  double lw_min, lw_max;           /* length / width */
  double tgrad_max;                /* samples per m, uniform in [-max, max] */
  double t0_center, t0_halfwidth;  /* samples */
  /* gamma / hadron draws */
  double e_min, e_max;             /* TeV, log-uniform */
  double size_per_tev;             /* p.e. per TeV for gammas */
  double hadron_fraction;          /* probability that an image is a hadron */
  double had_width_min, had_width_max, had_lw_min, had_lw_max;
  int32_t had_blobs_max;
  int32_t pad_;
} dl0sim_draw_cfg;

static double log_uniform(ph_stream* s, double lo, double hi) {
  return exp(log(lo) + (log(hi) - log(lo)) * ph_uniform(s));
}

static void draw_cog(ph_stream* s, double rmax, float* cx, float* cy) {
  double r = rmax * sqrt(ph_uniform(s));
  double th = 2.0 * DL0_PI * ph_uniform(s);
  *cx = (float)(r * cos(th));
  *cy = (float)(r * sin(th));
}

static void draw_one_ellipse(ph_stream* s, const dl0sim_draw_cfg* c, dl0sim_shower* o, int b,
                             double size, double wmin, double wmax, double lwmin, double lwmax) {
  draw_cog(s, c->cog_rmax, &o->cog_x[b], &o->cog_y[b]);
  o->psi[b] = (float)(-DL0_PI / 2 + DL0_PI * ph_uniform(s));
  double w = wmin + (wmax - wmin) * ph_uniform(s);
  o->width[b] = (float)w;
  o->length[b] = (float)(w * (lwmin + (lwmax - lwmin) * ph_uniform(s)));
  o->size[b] = (float)size;
  o->t0[b] = (float)(c->t0_center + c->t0_halfwidth * (2.0 * ph_uniform(s) - 1.0));
  o->tgrad[b] = (float)(c->tgrad_max * (2.0 * ph_uniform(s) - 1.0));
}

static void shower_clear(dl0sim_shower* o) {
  memset(o, 0, sizeof(*o));
  o->src_x = NAN;
  o->src_y = NAN;
}

/* Plain single-ellipse images (one camera type; the plain-method configurations). */
void dl0sim_draw_ellipses(const dl0sim_draw_cfg* c, uint64_t seed, int64_t first_event, int64_t n,
                          dl0sim_shower* out) {
  for (int64_t i = 0; i < n; ++i) {
    ph_stream s;
    ph_init(&s, seed, (uint64_t)(first_event + i), 0xFFFFFFu, 1);
    dl0sim_shower* o = &out[i];
    shower_clear(o);
    o->n_blob = 1;
    o->kind = 0;
    double size = log_uniform(&s, c->size_min, c->size_max);
    draw_one_ellipse(&s, c, o, 0, size, c->width_min, c->width_max, c->lw_min, c->lw_max);
  }
}

/* Gamma (one narrow ellipse, size proportional to energy) or hadron (1..k broad
 * blobs sharing a log-uniform total size split by a flat Dirichlet). */
void dl0sim_draw_gamma_hadron(const dl0sim_draw_cfg* c, uint64_t seed, int64_t first_event, int64_t n,
                              dl0sim_shower* out) {
  for (int64_t i = 0; i < n; ++i) {
    ph_stream s;
    ph_init(&s, seed, (uint64_t)(first_event + i), 0xFFFFFFu, 2);
    dl0sim_shower* o = &out[i];
    shower_clear(o);
    double e = log_uniform(&s, c->e_min, c->e_max);
    o->energy_tev = (float)e;
    if (ph_uniform(&s) >= c->hadron_fraction) {
      o->kind = 1;
      o->n_blob = 1;
      draw_one_ellipse(&s, c, o, 0, c->size_per_tev * e, c->width_min, c->width_max, c->lw_min, c->lw_max);
    } else {
      o->kind = 2;
      int nb = 1 + (int)(ph_uniform(&s) * c->had_blobs_max);
      if (nb > c->had_blobs_max) nb = c->had_blobs_max;
      if (nb > DL0_MAX_BLOB) nb = DL0_MAX_BLOB;
      o->n_blob = nb;
      double total = log_uniform(&s, c->size_per_tev * c->e_min, c->size_per_tev * c->e_max);
      double g[DL0_MAX_BLOB], gs = 0;
      for (int b = 0; b < nb; ++b) { g[b] = -log(ph_uniform(&s)); gs += g[b]; }
      for (int b = 0; b < nb; ++b)
        draw_one_ellipse(&s, c, o, b, total * g[b] / gs, c->had_width_min, c->had_width_max,
                         c->had_lw_min, c->had_lw_max);
    }
  }
}

/*
 * Array events: multiplicity uniform in [mult_min, mult_max], telescope types
 * i.i.d. with the given weights, one source point per array event (nominal
 * frame, radians, uniform in a disk of radius src_rmax).  Each telescope image
 * is an ellipse whose major axis points at the source image f_type * src.
 * Outputs: evt_tel_off[n_evt + 1], tel_type[n_tel_cap], showers[n_tel_cap],
 * src_nominal[n_evt][2].  Returns the number of telescopes, or -1 if the
 * capacity is too small.
 */
int64_t dl0sim_draw_array(const dl0sim_draw_cfg* c, uint64_t seed, int64_t first_event, int64_t n_evt,
                          int32_t mult_min, int32_t mult_max, int32_t n_types, const double* type_weight,
                          const double* focal_m, double src_rmax, int64_t n_tel_cap, int64_t* evt_tel_off,
                          int32_t* tel_type, dl0sim_shower* showers, double* src_nominal) {
  double wsum = 0;
  for (int t = 0; t < n_types; ++t) wsum += type_weight[t];
  int64_t nt = 0;
  evt_tel_off[0] = 0;
  for (int64_t e = 0; e < n_evt; ++e) {
    ph_stream s;
    ph_init(&s, seed, (uint64_t)(first_event + e), 0xFFFFFFu, 3);
    int32_t m = mult_min + (int32_t)(ph_uniform(&s) * (double)(mult_max - mult_min + 1));
    if (m > mult_max) m = mult_max;
    double r = src_rmax * sqrt(ph_uniform(&s)), th = 2.0 * DL0_PI * ph_uniform(&s);
    double sx = r * cos(th), sy = r * sin(th);
    src_nominal[2 * e] = sx;
    src_nominal[2 * e + 1] = sy;
    if (nt + m > n_tel_cap) return -1;
    for (int32_t k = 0; k < m; ++k) {
      ph_stream ts;
      ph_init(&ts, seed, (uint64_t)(first_event + e), (uint32_t)k, 4);
      double u = ph_uniform(&ts) * wsum, acc = 0;
      int32_t ty = n_types - 1;
      for (int t = 0; t < n_types; ++t) { acc += type_weight[t]; if (u < acc) { ty = t; break; } }
      tel_type[nt] = ty;
      dl0sim_shower* o = &showers[nt];
      shower_clear(o);
      o->n_blob = 1;
      double size = log_uniform(&ts, c->size_min, c->size_max);
      draw_one_ellipse(&ts, c, o, 0, size, c->width_min, c->width_max, c->lw_min, c->lw_max);
      double scx = focal_m[ty] * sx, scy = focal_m[ty] * sy;
      o->src_x = (float)scx;
      o->src_y = (float)scy;
      double dx = (double)o->cog_x[0] - scx, dy = (double)o->cog_y[0] - scy;
      double psi = atan2(dy, dx);
      if (psi > DL0_PI / 2) psi -= DL0_PI;
      if (psi <= -DL0_PI / 2) psi += DL0_PI;
      o->psi[0] = (float)psi;
      ++nt;
    }
    evt_tel_off[e + 1] = nt;
  }
  return nt;
}

/* ------------------------------------------------------------------ */
/* Rendering                                                            */
/* ------------------------------------------------------------------ */
typedef struct dl0sim_render_cfg {
  int32_t n_pix, n_pix_pad, n_samp, n_gain;
  int32_t hg_clip, lg_clip;       /* ADC ceilings (4095 / 65535) */
  int32_t n_threads, pad_;
  double noise_sigma;             /* ADC, independent per gain and sample */
  double nsb_rate;                /* p.e. per sample */
  double pulse_sigma;             /* samples */
  double pix_area;                /* m^2 */
  /* charge-image mode only */
  double image_window;            /* samples integrated by the extractor model */
} dl0sim_render_cfg;

/* Expected Cherenkov p.e. of blob b in a pixel at (x, y): size * area * N2. */
static double blob_mu(const dl0sim_shower* sh, int b, double area, double x, double y, double* l_out) {
  double c = cos((double)sh->psi[b]), s = sin((double)sh->psi[b]);
  double dx = x - sh->cog_x[b], dy = y - sh->cog_y[b];
  double l = dx * c + dy * s, w = -dx * s + dy * c;
  double L = sh->length[b], W = sh->width[b];
  *l_out = l;
  double z = 0.5 * (l * l / (L * L) + w * w / (W * W));
  if (z > 60.0) return 0.0;
  return (double)sh->size[b] * area * exp(-z) / (2.0 * DL0_PI * L * W);
}

typedef struct {
  const dl0sim_render_cfg* cfg;
  const float* x;
  const float* y;
  const float* base_ped;   /* [G][N] electronic pedestal, ADC */
  const float* adc_per_pe; /* [G][N] */
  const dl0sim_shower* showers;
  const uint64_t* event_ids;
  uint64_t seed;
  int64_t n;
  uint16_t* out;
  int32_t* out_d;          /* charge-image mode */
  float* out_t;
  float* out_npe;          /* optional [n][N] true photo-electrons */
  int64_t e_begin, e_end;
} render_job;

static void render_trace_event(const render_job* J, int64_t e) {
  const dl0sim_render_cfg* C = J->cfg;
  const int N = C->n_pix, Np = C->n_pix_pad, T = C->n_samp, G = C->n_gain;
  const dl0sim_shower* sh = &J->showers[e];
  uint16_t* ev = J->out + (size_t)e * (size_t)G * T * Np;
  memset(ev, 0, sizeof(uint16_t) * (size_t)G * T * Np);
  double* sig = (double*)malloc(sizeof(double) * (size_t)T);
  int32_t* nsb = (int32_t*)malloc(sizeof(int32_t) * (size_t)T);
  uint64_t eid = J->event_ids ? J->event_ids[e] : (uint64_t)e;
  const double inv_s2pi = 1.0 / (C->pulse_sigma * sqrt(2.0 * DL0_PI));
  for (int i = 0; i < N; ++i) {
    ph_stream ps;
    ph_init(&ps, J->seed, eid, (uint32_t)i, 5);
    for (int k = 0; k < T; ++k) sig[k] = 0.0;
    double npe_tot = 0;
    for (int b = 0; b < sh->n_blob; ++b) {
      double l;
      double mu = blob_mu(sh, b, C->pix_area, J->x[i], J->y[i], &l);
      int64_t npe = ph_poisson(&ps, mu);
      if (npe == 0) continue;
      npe_tot += (double)npe;
      double tp = (double)sh->t0[b] + (double)sh->tgrad[b] * l;
      int k0 = (int)floor(tp - 7.0 * C->pulse_sigma), k1 = (int)ceil(tp + 7.0 * C->pulse_sigma);
      if (k0 < 0) k0 = 0;
      if (k1 > T - 1) k1 = T - 1;
      for (int k = k0; k <= k1; ++k) {
        double z = ((double)k - tp) / C->pulse_sigma;
        sig[k] += (double)npe * exp(-0.5 * z * z) * inv_s2pi;
      }
    }
    if (J->out_npe) J->out_npe[(size_t)e * N + i] = (float)npe_tot;
    for (int k = 0; k < T; ++k) nsb[k] = (int32_t)ph_poisson(&ps, C->nsb_rate);
    for (int g = 0; g < G; ++g) {
      ph_stream ns;
      ph_init(&ns, J->seed, eid, (uint32_t)i, 6 + g);
      double a = J->adc_per_pe[g * N + i], p0 = J->base_ped[g * N + i];
      int clip = (g == 0) ? C->hg_clip : C->lg_clip;
      uint16_t* col = ev + (size_t)g * T * Np + i;
      for (int k = 0; k < T; k += 2) {
        double z0, z1;
        ph_normal2(&ns, &z0, &z1);
        for (int h = 0; h < 2 && k + h < T; ++h) {
          double v = p0 + a * (sig[k + h] + (double)nsb[k + h]) + C->noise_sigma * (h ? z1 : z0);
          v = nearbyint(v);
          if (v < 0) v = 0;
          if (v > clip) v = clip;
          col[(size_t)(k + h) * Np] = (uint16_t)v;
        }
      }
    }
  }
  free(nsb);
  free(sig);
}

/*
 * Charge-domain image: per pixel q = Cherenkov p.e. + (NSB p.e. in a window of
 * image_window samples, minus its mean) + electronic noise of the window, and
 * D = nearest integer of 256 * adc_per_pe * q (the Q8 calibrated-charge units
 * of the reconstruction).  t = pulse arrival time (+ jitter) for Cherenkov
 * pixels, uniform over the trace otherwise.  Gain 0 only.
 */
static void render_image_event(const render_job* J, int64_t e) {
  const dl0sim_render_cfg* C = J->cfg;
  const int N = C->n_pix, T = C->n_samp;
  const dl0sim_shower* sh = &J->showers[e];
  uint64_t eid = J->event_ids ? J->event_ids[e] : (uint64_t)e;
  const double wn = C->image_window;
  for (int i = 0; i < N; ++i) {
    ph_stream ps;
    ph_init(&ps, J->seed, eid, (uint32_t)i, 9);
    double npe_tot = 0, tsum = 0;
    for (int b = 0; b < sh->n_blob; ++b) {
      double l;
      double mu = blob_mu(sh, b, C->pix_area, J->x[i], J->y[i], &l);
      int64_t npe = ph_poisson(&ps, mu);
      if (npe == 0) continue;
      npe_tot += (double)npe;
      tsum += (double)npe * ((double)sh->t0[b] + (double)sh->tgrad[b] * l);
    }
    double a = J->adc_per_pe[i];
    double nsb = (double)ph_poisson(&ps, wn * C->nsb_rate) - wn * C->nsb_rate;
    double q = npe_tot + nsb + C->noise_sigma * sqrt(wn) / a * ph_normal(&ps);
    J->out_d[(size_t)e * N + i] = (int32_t)nearbyint(256.0 * a * q);
    double t;
    if (npe_tot > 0) t = tsum / npe_tot + ph_normal(&ps) * 0.5 / sqrt(npe_tot);
    else t = (double)(T - 1) * ph_uniform(&ps);
    J->out_t[(size_t)e * N + i] = (float)t;
    if (J->out_npe) J->out_npe[(size_t)e * N + i] = (float)npe_tot;
  }
}

static void* render_worker(void* arg) {
  render_job* J = (render_job*)arg;
  for (int64_t e = J->e_begin; e < J->e_end; ++e) {
    if (J->out) render_trace_event(J, e);
    else render_image_event(J, e);
  }
  return NULL;
}

static void run_jobs(render_job* base, int n_threads) {
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  if ((int64_t)n_threads > base->n) n_threads = (int)(base->n > 0 ? base->n : 1);
  pthread_t th[256];
  render_job jobs[256];
  for (int t = 0; t < n_threads; ++t) {
    jobs[t] = *base;
    jobs[t].e_begin = base->n * t / n_threads;
    jobs[t].e_end = base->n * (t + 1) / n_threads;
  }
  for (int t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, render_worker, &jobs[t]);
  render_worker(&jobs[0]);
  for (int t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
}

/*
 * Render n camera events of one camera type into out (uint16 [n][G][T][Npad]).
 * event_ids (nullable) gives the counter event index of each shower; otherwise
 * the position in the array is used.  npe_out (nullable): [n][N] true p.e.
 */
void dl0sim_render_traces(const dl0sim_render_cfg* cfg, const float* x, const float* y, const float* base_ped,
                          const float* adc_per_pe, const dl0sim_shower* showers, const uint64_t* event_ids,
                          uint64_t seed, int64_t n, uint16_t* out, float* npe_out) {
  render_job J;
  memset(&J, 0, sizeof(J));
  J.cfg = cfg; J.x = x; J.y = y; J.base_ped = base_ped; J.adc_per_pe = adc_per_pe;
  J.showers = showers; J.event_ids = event_ids; J.seed = seed; J.n = n; J.out = out; J.out_npe = npe_out;
  run_jobs(&J, cfg->n_threads);
}

/* Render n charge-domain images: D [n][N] int32 (Q8 units), t [n][N] float. */
void dl0sim_render_images(const dl0sim_render_cfg* cfg, const float* x, const float* y, const float* adc_per_pe,
                          const dl0sim_shower* showers, const uint64_t* event_ids, uint64_t seed, int64_t n,
                          int32_t* out_d, float* out_t, float* npe_out) {
  render_job J;
  memset(&J, 0, sizeof(J));
  J.cfg = cfg; J.x = x; J.y = y; J.adc_per_pe = adc_per_pe;
  J.showers = showers; J.event_ids = event_ids; J.seed = seed; J.n = n;
  J.out_d = out_d; J.out_t = out_t; J.out_npe = npe_out;
  run_jobs(&J, cfg->n_threads);
}

/* Raw Philox block, exported so tests can check the generator against the
 * published known-answer vectors. */
void dl0sim_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  ph_ctr c = {{ctr[0], ctr[1], ctr[2], ctr[3]}};
  ph_ctr r = philox4x32_10(c, key[0], key[1]);
  memcpy(out, r.v, sizeof(r.v));
}

int dl0sim_shower_size(void) { return (int)sizeof(dl0sim_shower); }

/* ------------------------------------------------------------------ */
/* DL0 telemetry packets                                                */
/*                                                                      */
/* The project's packet format for camera events on the byte stream    */
/* between the event builder and the analysis (in the style of space   */
/* telemetry source packets; every multi-byte field big-endian):       */
/*   0  u16  packet id: version 0 (3 b) | type 0 (1 b) | secondary     */
/*           header 1 (1 b) | APID = telescope id (11 b)                */
/*   2  u16  sequence control: flags 0b11 (unsegmented) | count (14 b) */
/*   4  u32  packet data length = total length - 9                     */
/*   8  u8   0x10   9 u8 service 210   10 u8 subtype 1                 */
/*  11  u8   camera type   12 u32 coarse time   16 u16 fine time       */
/*  18  u16  n_pix   20 u16 n_samp   22 u8 n_gain   23 u8 spare (0)    */
/*  24  u64  event number                                               */
/*  32  u16  samples [G][T][N] (no padding)                            */
/*  end u16  CRC-16 (poly 0x1021, init 0xFFFF) of every byte before it */
/* ------------------------------------------------------------------ */
static uint16_t crc_table_gen[256];
static int crc_table_ready = 0;

static void crc_table_init(void) {
  for (int i = 0; i < 256; ++i) {
    uint16_t r = (uint16_t)(i << 8);
    for (int k = 0; k < 8; ++k) r = (uint16_t)((r & 0x8000) ? (r << 1) ^ 0x1021 : (r << 1));
    crc_table_gen[i] = r;
  }
  crc_table_ready = 1;
}

uint16_t dl0sim_crc16(const uint8_t* p, int64_t n) {
  if (!crc_table_ready) crc_table_init();
  uint16_t c = 0xFFFF;
  for (int64_t i = 0; i < n; ++i) c = (uint16_t)((c << 8) ^ crc_table_gen[((c >> 8) ^ p[i]) & 0xFF]);
  return c;
}

static void put16(uint8_t* p, uint32_t v) { p[0] = (uint8_t)(v >> 8); p[1] = (uint8_t)v; }
static void put32(uint8_t* p, uint32_t v) { put16(p, v >> 16); put16(p + 2, v); }

/* One packet per camera event.  meta [n][8] int64: camera type, n_pix,
 * n_samp, n_gain, Npad, element offset of the event in blob, APID,
 * sequence count; evno [n], coarse [n] (u32), fine [n] (u16); out_off [n]
 * byte offset of each packet in out (the caller lays them out). */
void dl0sim_serialize_packets(int64_t n, const int64_t* meta, const uint64_t* evno, const uint32_t* coarse,
                              const uint16_t* fine, const uint16_t* blob, const int64_t* out_off, uint8_t* out) {
  if (!crc_table_ready) crc_table_init();
  for (int64_t e = 0; e < n; ++e) {
    const int64_t* m = meta + 8 * e;
    const int ty = (int)m[0], N = (int)m[1], T = (int)m[2], G = (int)m[3], Np = (int)m[4];
    const uint16_t* ev = blob + m[5];
    uint8_t* p = out + out_off[e];
    const int64_t body = 2LL * G * T * N, total = 32 + body + 2;
    put16(p, (1u << 11) | ((uint32_t)m[6] & 0x7FFu));
    put16(p + 2, (3u << 14) | ((uint32_t)m[7] & 0x3FFFu));
    put32(p + 4, (uint32_t)(total - 9));
    p[8] = 0x10; p[9] = 210; p[10] = 1; p[11] = (uint8_t)ty;
    put32(p + 12, coarse[e]);
    put16(p + 16, fine[e]);
    put16(p + 18, (uint32_t)N);
    put16(p + 20, (uint32_t)T);
    p[22] = (uint8_t)G; p[23] = 0;
    put32(p + 24, (uint32_t)(evno[e] >> 32));
    put32(p + 28, (uint32_t)evno[e]);
    uint8_t* q = p + 32;
    for (int g = 0; g < G; ++g)
      for (int k = 0; k < T; ++k)
        for (int i = 0; i < N; ++i, q += 2) put16(q, ev[((int64_t)g * T + k) * Np + i]);
    put16(p + 32 + body, dl0sim_crc16(p, 32 + body));
  }
}
