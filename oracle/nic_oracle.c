/*
 * FP64 CPU oracle for the training step of a hash-encoded attenuation field for sparse-view
 * cone-beam CT ("NeRF-based CBCT Reconstruction needs Normalization and Initialization",
 * Xu et al., arXiv 2506.19742).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct reference of what the
 * GPU path computes.  Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant generator with the HIP library; the two
 * agree only because both follow the same definitions, listed below with the passage each follows.
 *
 * Arithmetic is FP64 throughout, except where the method lets floating point decide an integer:
 * the normalised sample position handed to the hash encoder is an FP32 value and the cell of a
 * level is floor(fl32(x * N_l)), so both sides take that decision in the same (FP32) precision.
 * The sampling arithmetic that produces that FP32 position is a fixed sequence of FP64 operations
 * (this file is compiled with -ffp-contract=off so no multiply-add is fused).
 *
 * Definitions (paper passage, then the reading taken where the paper is silent):
 *  - Rendering: A = -ln(I/I0) = sum_i mu_i * delta_i along a ray (Sec. 2.2, Eq. 1).  Samples are
 *    stratified: N equal bins of the ray's segment inside the volume box, one jittered sample per
 *    bin, delta_i = bin length (reading: equal steps with stratified jitter).
 *  - Pixel loss: mean over the R rays of |A_gt - sum_i mu_i delta_i| (Sec. 2.5, Eq. 3; reading:
 *    mean rather than sum).
 *  - Field: multiresolution hash encoding (the paper cites Instant-NGP, Mueller et al. 2022, and does
 *    not restate it; Sec. 1) -> LayerNorm between encoder and network (the "Normalized Hash
 *    Encoder", Sec. 1 and Sec. 2.3; the formula is announced but missing, reading: per-point
 *    LayerNorm over the L*F channels with biased variance, eps and learnable gain/bias) -> MLP with
 *    ReLU hidden layers -> output activation (unstated; reading: mu = mu_max * sigmoid(y)).
 *  - Optimiser: Adam, lr 1e-3 (Sec. 3.1); beta = (0.9, 0.999), eps = 1e-8, dense update of every
 *    parameter every step (reading: PyTorch semantics).
 *  - Pre-training for Mapping Consistency Initialization: dense random points of the volume,
 *    voxel loss |mu_gt - M(x,y,z)| (Sec. 2.1, Sec. 2.4, Eq. 2; reading: mean over the batch).
 *  - Random draws of the training schedule (view order, ray pixels, jitter, initial values) use
 *    Philox4x32-10 (Salmon et al., SC'11) from its published definition.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_MAX_L 32
#define ORA_MAX_C 64
#define ORA_MAX_W 128
#define ORA_MAX_D 8

/* ------------------------------------------------------------------------------------------ */
/* Configuration                                                                               */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
  int32_t n_levels;        /* L */
  int32_t feats;           /* F */
  int32_t log2_table;      /* T = 2^log2_table entries per hashed level */
  int32_t base_res;        /* N_min */
  int32_t max_res;         /* N_max */
  int32_t depth;           /* D hidden layers */
  int32_t width;           /* W */
  int32_t out_act;         /* 0: mu_max*sigmoid, 1: identity, 2: softplus */
  int32_t layernorm;       /* 1: LayerNorm between encoder and network */
  int32_t masked;          /* 1: the encoder's channels are multiplied by mask[] before LayerNorm */
  double mu_max;
  double ln_eps;
  double mask[64];         /* channel mask (Sec. 2.3: noisy channels are masked), used when masked */
} ora_cfg;

typedef struct {
  double dso, dsd;          /* source-origin and source-detector distances (mm) */
  int32_t nu, nv;           /* detector columns, rows */
  double du, dv;            /* pixel pitch (mm) */
  double off_u, off_v;      /* detector offset (mm) */
  double vol[3];            /* box edge lengths (mm), centred at the origin */
} ora_geom;

typedef struct {
  int L, F, C, D, W;
  int32_t res[ORA_MAX_L];
  int32_t dense[ORA_MAX_L];
  int64_t off[ORA_MAX_L];
  int64_t size[ORA_MAX_L];
  int64_t n_entries;
  uint32_t T;
  /* offsets of the dense (LayerNorm + MLP) block, relative to its start */
  int64_t o_lng, o_lnb, o_W[ORA_MAX_D], o_b[ORA_MAX_D], o_wo, o_bo, n_dense;
} ora_layout;

/* Level resolutions of the multiresolution grid (Instant-NGP's geometric progression):
 * b = exp((ln N_max - ln N_min)/(L-1)), N_l = floor(N_min * b^l).  A level is dense (one entry per
 * grid vertex) when its (N_l+1)^3 vertices fit in T entries; otherwise it holds T hashed entries. */
static int make_layout(const ora_cfg* c, ora_layout* o) {
  memset(o, 0, sizeof(*o));
  if (c->n_levels < 1 || c->n_levels > ORA_MAX_L || c->feats < 1 || c->depth < 1 ||
      c->depth > ORA_MAX_D || c->width < 1 || c->width > ORA_MAX_W || c->log2_table < 1 ||
      c->log2_table > 30 || c->base_res < 1 || c->max_res < c->base_res)
    return -1;
  o->L = c->n_levels; o->F = c->feats; o->C = c->n_levels * c->feats; o->D = c->depth; o->W = c->width;
  if (o->C > ORA_MAX_C) return -1;
  o->T = 1u << c->log2_table;
  double b = (o->L > 1) ? exp((log((double)c->max_res) - log((double)c->base_res)) / (double)(o->L - 1)) : 1.0;
  int64_t off = 0;
  for (int l = 0; l < o->L; ++l) {
    double r = floor((double)c->base_res * pow(b, (double)l));
    o->res[l] = (int32_t)r;
    double nv = ((double)o->res[l] + 1.0) * ((double)o->res[l] + 1.0) * ((double)o->res[l] + 1.0);
    o->dense[l] = nv <= (double)o->T;
    o->size[l] = o->dense[l] ? (int64_t)nv : (int64_t)o->T;
    o->off[l] = off;
    off += o->size[l];
  }
  o->n_entries = off;
  int64_t p = 0;
  o->o_lng = p; p += o->C;
  o->o_lnb = p; p += o->C;
  for (int k = 0; k < o->D; ++k) {
    int in = (k == 0) ? o->C : o->W;
    o->o_W[k] = p; p += (int64_t)o->W * in;
    o->o_b[k] = p; p += o->W;
  }
  o->o_wo = p; p += o->W;
  o->o_bo = p; p += 1;
  o->n_dense = p;
  return 0;
}

int ora_levels(const ora_cfg* c, int32_t* res, int32_t* dense, int64_t* off, int64_t* size,
               int64_t* n_entries) {
  ora_layout o;
  if (make_layout(c, &o)) return -1;
  for (int l = 0; l < o.L; ++l) { res[l] = o.res[l]; dense[l] = o.dense[l]; off[l] = o.off[l]; size[l] = o.size[l]; }
  *n_entries = o.n_entries;
  return 0;
}

/* Number of parameters: table (n_entries * F) followed by the dense block
 * [ln_gain C][ln_bias C] then per hidden layer k [W_k (W x in_k, row = output unit)][b_k W]
 * then [w_out W][b_out 1]. */
int64_t ora_n_params(const ora_cfg* c, int64_t* n_table, int64_t* n_dense) {
  ora_layout o;
  if (make_layout(c, &o)) return -1;
  if (n_table) *n_table = o.n_entries * o.F;
  if (n_dense) *n_dense = o.n_dense;
  return o.n_entries * o.F + o.n_dense;
}

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) */
/* ------------------------------------------------------------------------------------------ */

void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static uint32_t philox_word0(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  ora_philox4x32_10(ctr, key, out);
  return out[0];
}

/* 24-bit uniform in [0,1): exactly representable in FP32 and FP64. */
static double u24(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

/* Stream ids placed in the fourth counter word. */
enum { ORA_S_JITTER = 1, ORA_S_RAYS = 2, ORA_S_VIEWS = 3, ORA_S_TABLE = 4, ORA_S_MLP = 5, ORA_S_POINTS = 6 };

/* Jitter of sample i of ray slot j at step t. */
double ora_jitter(uint64_t seed, uint32_t t, uint32_t j, uint32_t i) {
  return u24(philox_word0(seed, i, j, t, ORA_S_JITTER));
}

/* Keyed bijection on [0, 2^(2h)): a four-round balanced Feistel network (Luby and Rackoff) whose
 * round function is the first Philox word of (right half, round, step, stream). */
static uint32_t feistel(uint64_t seed, uint32_t t, int h, uint32_t x) {
  uint32_t mask = (h >= 32) ? 0xFFFFFFFFu : ((1u << h) - 1u);
  uint32_t L = (x >> h) & mask, R = x & mask;
  for (uint32_t rnd = 0; rnd < 4; ++rnd) {
    uint32_t f = philox_word0(seed, R, rnd, t, ORA_S_RAYS) & mask;
    uint32_t nL = R, nR = L ^ f;
    L = nL; R = nR;
  }
  return (L << h) | R;
}

static int half_bits(int64_t n_pix) {
  int bits = 0;
  while (((int64_t)1 << bits) < n_pix) ++bits;
  if (bits & 1) ++bits;
  if (bits < 2) bits = 2;
  return bits / 2;
}

/* Pixel of ray slot j at step t: the Feistel bijection restricted to [0, n_pix) by cycle walking.
 * Distinct slots give distinct pixels (uniform sampling without replacement within a step). */
int32_t ora_ray_pixel(uint64_t seed, uint32_t t, int64_t n_pix, uint32_t j) {
  int h = half_bits(n_pix);
  uint32_t y = feistel(seed, t, h, j);
  while ((int64_t)y >= n_pix) y = feistel(seed, t, h, y);
  return (int32_t)y;
}

/* View of step t: views are visited in a fresh random order each epoch of V steps; the order of
 * epoch e sorts views by Philox key (ties by view index). */
int32_t ora_view_for_step(uint64_t seed, uint32_t t, int32_t V) {
  uint32_t e = t / (uint32_t)V, pos = t % (uint32_t)V;
  /* the view at position pos is the one with exactly pos views ordered before it */
  for (int32_t v = 0; v < V; ++v) {
    uint32_t kv = philox_word0(seed, (uint32_t)v, e, 0, ORA_S_VIEWS);
    uint32_t before = 0;
    for (int32_t w = 0; w < V; ++w) {
      uint32_t kw = philox_word0(seed, (uint32_t)w, e, 0, ORA_S_VIEWS);
      if (kw < kv || (kw == kv && w < v)) ++before;
    }
    if (before == pos) return v;
  }
  return -1;
}

/* Ray slots and jitter of step t as arrays (used to compare the GPU's own draws bit for bit). */
void ora_draw_rays(uint64_t seed, uint32_t t, int64_t n_pix, int32_t R, int32_t N, int32_t* pix,
                   float* jitter) {
  for (int32_t j = 0; j < R; ++j) {
    pix[j] = ora_ray_pixel(seed, t, n_pix, (uint32_t)j);
    for (int32_t i = 0; i < N; ++i) jitter[(int64_t)j * N + i] = (float)ora_jitter(seed, t, (uint32_t)j, (uint32_t)i);
  }
}

/* Points of a voxel-loss step (pre-training, Eq. 2): point p of step t takes its three normalised
 * coordinates from the first three words of the Philox block (p, t, 0, stream). */
void ora_voxel_points(uint64_t seed, uint32_t t, int32_t n, float* xn) {
  for (int32_t p = 0; p < n; ++p) {
    uint32_t ctr[4] = {(uint32_t)p, t, 0u, ORA_S_POINTS};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    ora_philox4x32_10(ctr, key, out);
    for (int k = 0; k < 3; ++k) xn[3 * (int64_t)p + k] = (float)u24(out[k]);
  }
}

/* Initial parameters: table entries uniform in [-1e-4, 1e-4); linear layers uniform in
 * [-1/sqrt(fan_in), 1/sqrt(fan_in)) (the usual default for linear layers; the paper states no
 * initialisation); LayerNorm gain 1 and bias 0. */
void ora_init_params(const ora_cfg* c, uint64_t seed, double* params) {
  ora_layout o;
  if (make_layout(c, &o)) return;
  int64_t nt = o.n_entries * o.F;
  for (int64_t e = 0; e < nt; ++e) {
    double u = u24(philox_word0(seed, (uint32_t)e, (uint32_t)((uint64_t)e >> 32), 0, ORA_S_TABLE));
    params[e] = (2.0 * u - 1.0) * 1e-4;
  }
  double* d = params + nt;
  for (int i = 0; i < o.C; ++i) { d[o.o_lng + i] = 1.0; d[o.o_lnb + i] = 0.0; }
  for (int l = 0; l <= o.D; ++l) {
    /* layer l < D is hidden layer l (weights then biases); l == D is the output unit */
    int64_t first = (l < o.D) ? o.o_W[l] : o.o_wo;
    int64_t last = (l < o.D) ? o.o_b[l] + o.W : o.o_bo + 1;
    int fan_in = (l == 0) ? o.C : o.W;
    for (int64_t k = first; k < last; ++k) {
      double u = u24(philox_word0(seed, (uint32_t)k, 0, 0, ORA_S_MLP));
      d[k] = (2.0 * u - 1.0) / sqrt((double)fan_in);
    }
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Multiresolution hash encoding (Instant-NGP, cited in Sec. 1)                                */
/* ------------------------------------------------------------------------------------------ */

/* Index of grid vertex v within level l.  Dense levels: v0 + (N_l+1)(v1 + (N_l+1) v2).
 * Hashed levels: (v0*1 XOR v1*2654435761 XOR v2*805459861) mod 2^32, then mod T. */
uint32_t ora_vertex_index(const ora_cfg* c, int l, uint32_t v0, uint32_t v1, uint32_t v2) {
  ora_layout o;
  if (make_layout(c, &o)) return 0xFFFFFFFFu;
  if (o.dense[l]) {
    uint64_t s = (uint64_t)o.res[l] + 1u;
    return (uint32_t)((uint64_t)v0 + s * ((uint64_t)v1 + s * (uint64_t)v2));
  }
  uint32_t h = (v0 * 1u) ^ (v1 * 2654435761u) ^ (v2 * 805459861u);
  return h & (o.T - 1u);
}

/* Per level: cell g = min(floor(fl32(x*N_l)), N_l-1) per axis, fraction f = pos - g, eight corners
 * c = c0 + 2 c1 + 4 c2 at vertex g + c with trilinear weight prod_d (c_d ? f_d : 1 - f_d). */
static void level_corners(const ora_cfg* c, const ora_layout* o, int l, const float x[3],
                          int64_t entry[8], double w[8]) {
  uint32_t g[3];
  double f[3];
  for (int d = 0; d < 3; ++d) {
    float pos = x[d] * (float)o->res[l];     /* one FP32 multiply, round to nearest even */
    float fl = floorf(pos);
    int32_t gi = (int32_t)fl;
    if (gi > o->res[l] - 1) gi = o->res[l] - 1;
    if (gi < 0) gi = 0;
    g[d] = (uint32_t)gi;
    f[d] = (double)(pos - (float)gi);        /* exact in FP32 */
  }
  for (int k = 0; k < 8; ++k) {
    int c0 = k & 1, c1 = (k >> 1) & 1, c2 = (k >> 2) & 1;
    uint32_t local = ora_vertex_index(c, l, g[0] + c0, g[1] + c1, g[2] + c2);
    entry[k] = o->off[l] + (int64_t)local;
    w[k] = (c0 ? f[0] : 1.0 - f[0]) * (c1 ? f[1] : 1.0 - f[1]) * (c2 ? f[2] : 1.0 - f[2]);
  }
}

/* enc[p][l*F + f] = sum over corners of w_c * table[entry_c][f].  Optionally also returns the
 * global entry index (level offset included) and the weight of every corner. */
void ora_encode(const ora_cfg* c, const double* table, const float* xn, int64_t n, double* enc,
                uint32_t* idx, double* wts) {
  ora_layout o;
  if (make_layout(c, &o)) return;
  for (int64_t p = 0; p < n; ++p) {
    for (int l = 0; l < o.L; ++l) {
      int64_t entry[8];
      double w[8];
      level_corners(c, &o, l, xn + 3 * p, entry, w);
      for (int f = 0; f < o.F; ++f) {
        double s = 0.0;
        for (int k = 0; k < 8; ++k) s += w[k] * table[entry[k] * o.F + f];
        enc[p * o.C + l * o.F + f] = s;
      }
      for (int k = 0; k < 8; ++k) {
        if (idx) idx[(p * o.L + l) * 8 + k] = (uint32_t)entry[k];
        if (wts) wts[(p * o.L + l) * 8 + k] = w[k];
      }
    }
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Field: encode -> LayerNorm (Sec. 2.3) -> MLP -> output activation                            */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
  int64_t entry[ORA_MAX_L][8];
  double w[ORA_MAX_L][8];
  double enc[ORA_MAX_C];
  double xhat[ORA_MAX_C];
  double z[ORA_MAX_C];
  double mean, rstd;
  double a[ORA_MAX_D][ORA_MAX_W];
  double h[ORA_MAX_D][ORA_MAX_W];
  double y, mu;
} point_state;

/* Output activation (unstated in the paper).  0: mu = mu_max * sigmoid(y); 1: identity;
 * 2: softplus log(1 + e^y), taken as PyTorch's Softplus (beta 1, threshold 20): above the threshold
 * the output is y itself and its derivative exactly 1. */
static double act_fwd(const ora_cfg* c, double y) {
  if (c->out_act == 1) return y;
  if (c->out_act == 2) return (y > 20.0) ? y : log1p(exp(y));
  return c->mu_max / (1.0 + exp(-y));
}

static double act_grad(const ora_cfg* c, double y) {
  if (c->out_act == 1) return 1.0;
  if (c->out_act == 2) return (y > 20.0) ? 1.0 : 1.0 / (1.0 + exp(-y));
  double s = 1.0 / (1.0 + exp(-y));
  return c->mu_max * s * (1.0 - s);
}

static void features_forward(const ora_cfg* c, const ora_layout* o, const double* d, point_state* st);

static void point_forward(const ora_cfg* c, const ora_layout* o, const double* table, const double* d,
                          const float x[3], point_state* st) {
  for (int l = 0; l < o->L; ++l) {
    level_corners(c, o, l, x, st->entry[l], st->w[l]);
    for (int f = 0; f < o->F; ++f) {
      double s = 0.0;
      for (int k = 0; k < 8; ++k) s += st->w[l][k] * table[st->entry[l][k] * o->F + f];
      st->enc[l * o->F + f] = s;
    }
  }
  features_forward(c, o, d, st);
}

/* From the encoder output st->enc to mu: LayerNorm (Sec. 2.3), hidden layers, head, activation. */
static void features_forward(const ora_cfg* c, const ora_layout* o, const double* d, point_state* st) {
  /* Channel mask (Sec. 2.3): the network sees mask[i] * enc[i]; st->enc keeps the raw encoding. */
  double e[ORA_MAX_C];
  for (int i = 0; i < o->C; ++i) e[i] = c->masked ? c->mask[i] * st->enc[i] : st->enc[i];
  /* LayerNorm over the C channels of this point: biased variance, then gain and bias. */
  if (c->layernorm) {
    double m = 0.0;
    for (int i = 0; i < o->C; ++i) m += e[i];
    m /= (double)o->C;
    double v = 0.0;
    for (int i = 0; i < o->C; ++i) v += (e[i] - m) * (e[i] - m);
    v /= (double)o->C;
    double s = 1.0 / sqrt(v + c->ln_eps);
    st->mean = m; st->rstd = s;
    for (int i = 0; i < o->C; ++i) {
      st->xhat[i] = (e[i] - m) * s;
      st->z[i] = d[o->o_lng + i] * st->xhat[i] + d[o->o_lnb + i];
    }
  } else {
    st->mean = 0.0; st->rstd = 1.0;
    for (int i = 0; i < o->C; ++i) { st->xhat[i] = e[i]; st->z[i] = e[i]; }
  }
  /* Hidden layers: a_k = W_k h_{k-1} + b_k, h_k = max(a_k, 0). */
  const double* hin = st->z;
  int in = o->C;
  for (int k = 0; k < o->D; ++k) {
    const double* Wk = d + o->o_W[k];
    const double* bk = d + o->o_b[k];
    for (int u = 0; u < o->W; ++u) {
      double s = bk[u];
      for (int i = 0; i < in; ++i) s += Wk[(int64_t)u * in + i] * hin[i];
      st->a[k][u] = s;
      st->h[k][u] = s > 0.0 ? s : 0.0;
    }
    hin = st->h[k];
    in = o->W;
  }
  double y = d[o->o_bo];
  for (int u = 0; u < o->W; ++u) y += d[o->o_wo + u] * st->h[o->D - 1][u];
  st->y = y;
  st->mu = act_fwd(c, y);
}

/* Accumulates d(loss)/d(params) for one point given dmu = d(loss)/d(mu).  The hash table receives a
 * scatter-add over the 8 corners of every level (collisions add); there is no position gradient. */
static void point_backward(const ora_cfg* c, const ora_layout* o, const double* d, const point_state* st,
                           double dmu, double* gt, double* gd) {
  double dy = dmu * act_grad(c, st->y);
  double gh[ORA_MAX_W], ga[ORA_MAX_W], gin[ORA_MAX_W];
  for (int u = 0; u < o->W; ++u) {
    gd[o->o_wo + u] += dy * st->h[o->D - 1][u];
    gh[u] = dy * d[o->o_wo + u];
  }
  gd[o->o_bo] += dy;
  for (int k = o->D - 1; k >= 0; --k) {
    int in = (k == 0) ? o->C : o->W;
    const double* hprev = (k == 0) ? st->z : st->h[k - 1];
    const double* Wk = d + o->o_W[k];
    for (int u = 0; u < o->W; ++u) ga[u] = (st->a[k][u] > 0.0) ? gh[u] : 0.0;   /* ReLU'(0) = 0 */
    for (int u = 0; u < o->W; ++u) {
      gd[o->o_b[k] + u] += ga[u];
      for (int i = 0; i < in; ++i) gd[o->o_W[k] + (int64_t)u * in + i] += ga[u] * hprev[i];
    }
    for (int i = 0; i < in; ++i) {
      double s = 0.0;
      for (int u = 0; u < o->W; ++u) s += Wk[(int64_t)u * in + i] * ga[u];
      gin[i] = s;
    }
    for (int i = 0; i < in; ++i) gh[i] = gin[i];
  }
  /* gh now holds d(loss)/dz over the C channels. */
  double gx[ORA_MAX_C];
  if (c->layernorm) {
    double g[ORA_MAX_C], mg = 0.0, mgx = 0.0;
    for (int i = 0; i < o->C; ++i) {
      gd[o->o_lng + i] += gh[i] * st->xhat[i];
      gd[o->o_lnb + i] += gh[i];
      g[i] = d[o->o_lng + i] * gh[i];
      mg += g[i];
      mgx += g[i] * st->xhat[i];
    }
    mg /= (double)o->C;
    mgx /= (double)o->C;
    for (int i = 0; i < o->C; ++i) gx[i] = st->rstd * (g[i] - mg - st->xhat[i] * mgx);
  } else {
    for (int i = 0; i < o->C; ++i) gx[i] = gh[i];
  }
  if (c->masked)   /* back through the channel mask to the raw encoding */
    for (int i = 0; i < o->C; ++i) gx[i] *= c->mask[i];
  for (int l = 0; l < o->L; ++l)
    for (int k = 0; k < 8; ++k)
      for (int f = 0; f < o->F; ++f)
        gt[st->entry[l][k] * o->F + f] += st->w[l][k] * gx[l * o->F + f];
}

/* mu at n points (normalised FP32 coordinates).  Optional outputs: enc (raw encoding) and z
 * (LayerNorm output), both [n][C]. */
void ora_field(const ora_cfg* c, const double* params, const float* xn, int64_t n, double* mu,
               double* enc, double* z) {
  ora_layout o;
  if (make_layout(c, &o)) return;
  const double* dn = params + o.n_entries * o.F;
  point_state* st = (point_state*)malloc(sizeof(point_state));
  for (int64_t p = 0; p < n; ++p) {
    point_forward(c, &o, params, dn, xn + 3 * p, st);
    mu[p] = st->mu;
    if (enc) for (int i = 0; i < o.C; ++i) enc[p * o.C + i] = st->enc[i];
    if (z) for (int i = 0; i < o.C; ++i) z[p * o.C + i] = st->z[i];
  }
  free(st);
}

/* mu from given encoder outputs enc [n][C] (channel l*F + f): the feature-to-attenuation mapping
 * alone, as studied for fixed features in Fig. 3. */
void ora_field_from_features(const ora_cfg* c, const double* params, const double* enc, int64_t n,
                             double* mu) {
  ora_layout o;
  if (make_layout(c, &o)) return;
  const double* dn = params + o.n_entries * o.F;
  point_state* st = (point_state*)malloc(sizeof(point_state));
  for (int64_t p = 0; p < n; ++p) {
    for (int i = 0; i < o.C; ++i) st->enc[i] = enc[p * o.C + i];
    features_forward(c, &o, dn, st);
    mu[p] = st->mu;
  }
  free(st);
}

/* Gradient of sum_p dmu[p] * mu(x_p) with respect to all parameters (accumulated into grad). */
void ora_field_backward(const ora_cfg* c, const double* params, const float* xn, int64_t n,
                        const double* dmu, double* grad) {
  ora_layout o;
  if (make_layout(c, &o)) return;
  const double* dn = params + o.n_entries * o.F;
  point_state* st = (point_state*)malloc(sizeof(point_state));
  for (int64_t p = 0; p < n; ++p) {
    point_forward(c, &o, params, dn, xn + 3 * p, st);
    point_backward(c, &o, dn, st, dmu[p], grad, grad + o.n_entries * o.F);
  }
  free(st);
}

/* ------------------------------------------------------------------------------------------ */
/* Cone-beam rays and sampling (Sec. 2.2; Sec. 3.1 data)                                       */
/* ------------------------------------------------------------------------------------------ */

/* Circular orbit about z.  Source s = DSO (cos a, sin a, 0); detector centre
 * -(DSD - DSO)(cos a, sin a, 0); detector axes e_u = (-sin a, cos a, 0), e_v = (0, 0, 1).
 * Pixel (row r, column c) centre at u = ((c + 1/2) - nu/2) du + off_u, v = ((r + 1/2) - nv/2) dv
 * + off_v.  Ray x(t) = s + t (P - s), t in [0, 1], clipped to the box [-vol/2, vol/2] by the slab
 * method.  Returns 1 on a hit and fills s, d = P - s, [t0, t1] and the source-pixel length. */
static int ray_setup(const ora_geom* g, double ang, int32_t pix, double s[3], double d[3], double* t0,
                     double* t1, double* len) {
  double ca = cos(ang), sa = sin(ang);
  int32_t row = pix / g->nu, col = pix % g->nu;
  s[0] = g->dso * ca;
  s[1] = g->dso * sa;
  s[2] = 0.0;
  double back = g->dsd - g->dso;
  double dc0 = -(back * ca), dc1 = -(back * sa);
  double u = (((double)col + 0.5) - 0.5 * (double)g->nu) * g->du + g->off_u;
  double v = (((double)row + 0.5) - 0.5 * (double)g->nv) * g->dv + g->off_v;
  double P0 = dc0 + u * (-sa);
  double P1 = dc1 + u * ca;
  double P2 = v;
  d[0] = P0 - s[0];
  d[1] = P1 - s[1];
  d[2] = P2 - s[2];
  double lo = 0.0, hi = 1.0;
  for (int k = 0; k < 3; ++k) {
    double bl = -0.5 * g->vol[k], bh = 0.5 * g->vol[k];
    if (d[k] != 0.0) {
      double ta = (bl - s[k]) / d[k];
      double tb = (bh - s[k]) / d[k];
      double tn = ta < tb ? ta : tb;
      double tf = ta < tb ? tb : ta;
      if (tn > lo) lo = tn;
      if (tf < hi) hi = tf;
    } else if (s[k] < bl || s[k] > bh) {
      return 0;
    }
  }
  *t0 = lo;
  *t1 = hi;
  *len = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
  return hi > lo;
}

/* N stratified samples of one ray: bin dt = (t1 - t0)/N, t_i = t0 + (i + u_i) dt, step
 * delta = dt * |P - s| (mm).  Normalised coordinate per axis (x_k + vol_k/2) * (1/vol_k), clamped
 * to [0, 1], then rounded to FP32.  A ray that misses the box gets delta = 0 and no samples. */
int ora_ray_samples(const ora_geom* g, double ang, int32_t pix, int32_t N, const float* jitter,
                    float* xn, double* delta) {
  double s[3], d[3], t0, t1, len;
  int hit = ray_setup(g, ang, pix, s, d, &t0, &t1, &len);
  if (!hit) {
    *delta = 0.0;
    for (int64_t i = 0; i < 3 * (int64_t)N; ++i) xn[i] = 0.0f;
    return 0;
  }
  double dt = (t1 - t0) / (double)N;
  *delta = dt * len;
  for (int32_t i = 0; i < N; ++i) {
    double t = t0 + ((double)i + (double)jitter[i]) * dt;
    for (int k = 0; k < 3; ++k) {
      double x = s[k] + t * d[k];
      double xr = (x + 0.5 * g->vol[k]) * (1.0 / g->vol[k]);
      if (xr < 0.0) xr = 0.0;
      if (xr > 1.0) xr = 1.0;
      xn[3 * i + k] = (float)xr;
    }
  }
  return 1;
}

/* ------------------------------------------------------------------------------------------ */
/* Ray batch: Eq. (1) rendering, Eq. (3) L1 loss and the full backward pass                     */
/* ------------------------------------------------------------------------------------------ */

/* Host threads for ora_ray_batch (1 = serial).  Threads take contiguous ranges of rays; each
 * accumulates its gradient into a buffer of its own, and the buffers are added to the caller's
 * gradient in thread order, so a given thread count always gives the same sums.  The loss is summed
 * over rays in ray order whatever the thread count. */
static int g_threads = 1;

void ora_set_threads(int32_t n) { g_threads = n < 1 ? 1 : n; }

int32_t ora_get_threads(void) { return g_threads; }

/* One ray r of a batch: Eq. (1) sum over its samples into a_pred[r], its residual A - A_gt into
 * *res, and, when grad != NULL and the ray hits the box, the gradient of dA * A (dA from Eq. (3)
 * in mode 0, given in mode 1) accumulated into grad. */
static void ray_one(const ora_cfg* c, const ora_layout* o, const ora_geom* g, const double* params,
                    double angle, const float* proj_view, int32_t R, const int32_t* pix, int32_t N,
                    const float* jitter, int32_t mode, const double* dA_in, int32_t r, float* xn,
                    point_state* st, double* a_pred, double* res, double* grad) {
  const double* dn = params + o->n_entries * o->F;
  double delta;
  int hit = ora_ray_samples(g, angle, pix[r], N, jitter + (int64_t)r * N, xn, &delta);
  double A = 0.0;
  if (hit)
    for (int32_t i = 0; i < N; ++i) {
      point_forward(c, o, params, dn, xn + 3 * i, st);
      A += st->mu * delta;
    }
  a_pred[r] = A;
  const double rs = A - (double)proj_view[pix[r]];
  *res = rs;
  if (grad && hit) {
    double dA = (mode == 0) ? ((rs > 0.0) - (rs < 0.0)) / (double)R : dA_in[r];
    for (int32_t i = 0; i < N; ++i) {
      point_forward(c, o, params, dn, xn + 3 * i, st);
      point_backward(c, o, dn, st, dA * delta, grad, grad + o->n_entries * o->F);
    }
  }
}

/* Renders R rays of one view (pixel indices and per-sample jitter given) and, when grad != NULL,
 * accumulates the gradient.  mode 0: loss = mean_r |A_pred_r - A_gt_r| (Eq. 3) and
 * dA_r = sign(A_pred_r - A_gt_r)/R (sign(0) = 0); mode 1: dA is given (upstream gradient of
 * A_pred, for the autograd form) and the return value is 0.  proj is the view's image [nv][nu]. */
double ora_ray_batch(const ora_cfg* c, const ora_geom* g, const double* params, double angle,
                     const float* proj_view, int32_t R, const int32_t* pix, int32_t N,
                     const float* jitter, int32_t mode, const double* dA_in, double* a_pred,
                     double* grad) {
  ora_layout o;
  if (make_layout(c, &o)) return NAN;
  const int64_t np = o.n_entries * o.F + o.n_dense;
  int nth = g_threads < R ? g_threads : (R > 0 ? R : 1);
  double* res = (double*)malloc(sizeof(double) * (size_t)(R > 0 ? R : 1));
  double** bufs = NULL;
  if (grad && nth > 1) {
    bufs = (double**)calloc((size_t)nth, sizeof(double*));
    for (int t = 1; t < nth; ++t) {
      bufs[t] = (double*)calloc((size_t)np, sizeof(double));
      if (!bufs[t]) { nth = t; break; }   /* out of memory: fewer threads */
    }
  }
#pragma omp parallel num_threads(nth)
  {
#ifdef _OPENMP
    const int t = omp_get_thread_num();
#else
    const int t = 0;
#endif
    const int32_t r0 = (int32_t)((int64_t)R * t / nth), r1 = (int32_t)((int64_t)R * (t + 1) / nth);
    double* gt = (grad && t > 0) ? bufs[t] : grad;
    float* xn = (float*)malloc(sizeof(float) * 3 * (size_t)N);
    point_state* st = (point_state*)malloc(sizeof(point_state));
    for (int32_t r = r0; r < r1; ++r)
      ray_one(c, &o, g, params, angle, proj_view, R, pix, N, jitter, mode, dA_in, r, xn, st, a_pred,
              &res[r], gt);
    free(st);
    free(xn);
  }
  if (bufs) {
#pragma omp parallel for num_threads(nth) schedule(static)
    for (int64_t i = 0; i < np; ++i)
      for (int t = 1; t < nth; ++t) grad[i] += bufs[t][i];
    for (int t = 1; t < nth; ++t) free(bufs[t]);
    free(bufs);
  }
  double loss = 0.0;
  if (mode == 0)
    for (int32_t r = 0; r < R; ++r) loss += fabs(res[r]);
  free(res);
  return (mode == 0) ? loss / (double)R : 0.0;
}

/* ------------------------------------------------------------------------------------------ */
/* Adam (Kingma and Ba, Algorithm 1), dense over all parameters; lr from Sec. 3.1              */
/* ------------------------------------------------------------------------------------------ */

void ora_adam(double* p, const double* g, double* m, double* v, int64_t n, int64_t t, double lr,
              double b1, double b2, double eps) {
  double bc1 = 1.0 - pow(b1, (double)t);
  double bc2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / bc1;
    double vh = v[i] / bc2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ------------------------------------------------------------------------------------------ */
/* Full training steps with the schedule drawn from Philox (one view per step, Sec. 3.1)        */
/* ------------------------------------------------------------------------------------------ */

/* Runs n_steps steps starting at step index t_start (Adam step t_start + 1 first).  proj holds all
 * views [V][nv][nu]; angles [V].  losses[k] receives the loss of step k. */
int ora_train(const ora_cfg* c, const ora_geom* g, const double* angles, int32_t V, const float* proj,
              double* params, double* m, double* v, int64_t t_start, int32_t n_steps, int32_t R,
              int32_t N, uint64_t seed, double lr, double b1, double b2, double eps, double* losses) {
  int64_t np = ora_n_params(c, NULL, NULL);
  if (np < 0) return -1;
  int64_t n_pix = (int64_t)g->nu * g->nv;
  int32_t* pix = (int32_t*)malloc(sizeof(int32_t) * (size_t)R);
  float* jit = (float*)malloc(sizeof(float) * (size_t)R * (size_t)N);
  double* a = (double*)malloc(sizeof(double) * (size_t)R);
  double* grad = (double*)malloc(sizeof(double) * (size_t)np);
  for (int32_t k = 0; k < n_steps; ++k) {
    uint32_t t = (uint32_t)(t_start + k);
    int32_t view = ora_view_for_step(seed, t, V);
    ora_draw_rays(seed, t, n_pix, R, N, pix, jit);
    memset(grad, 0, sizeof(double) * (size_t)np);
    double L = ora_ray_batch(c, g, params, angles[view], proj + (int64_t)view * n_pix, R, pix, N, jit,
                             0, NULL, a, grad);
    if (losses) losses[k] = L;
    ora_adam(params, grad, m, v, np, (int64_t)t + 1, lr, b1, b2, eps);
  }
  free(pix); free(jit); free(a); free(grad);
  return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Volume rendering at voxel centres and PSNR                                                  */
/* ------------------------------------------------------------------------------------------ */

/* vol[z][y][x] = mu at the voxel centre ((x + 1/2)/nx, (y + 1/2)/ny, (z + 1/2)/nz) in normalised
 * coordinates (each computed in FP64 and rounded to FP32). */
void ora_render_volume(const ora_cfg* c, const double* params, int32_t nx, int32_t ny, int32_t nz,
                       double* vol) {
  ora_layout o;
  if (make_layout(c, &o)) return;
  point_state* st = (point_state*)malloc(sizeof(point_state));
  for (int32_t iz = 0; iz < nz; ++iz)
    for (int32_t iy = 0; iy < ny; ++iy)
      for (int32_t ix = 0; ix < nx; ++ix) {
        float x[3] = {(float)(((double)ix + 0.5) / (double)nx), (float)(((double)iy + 0.5) / (double)ny),
                      (float)(((double)iz + 0.5) / (double)nz)};
        point_forward(c, &o, params, params + o.n_entries * o.F, x, st);
        vol[((int64_t)iz * ny + iy) * nx + ix] = st->mu;
      }
  free(st);
}

/* PSNR = 10 log10(max(gt)^2 / MSE) over all voxels (peak = max of the ground truth). */
double ora_psnr(const double* gt, const double* pred, int64_t n) {
  double mx = -INFINITY, se = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (gt[i] > mx) mx = gt[i];
    double e = pred[i] - gt[i];
    se += e * e;
  }
  double mse = se / (double)n;
  if (mse == 0.0) return INFINITY;
  return 10.0 * log10(mx * mx / mse);
}

/* 3-D SSIM (Wang et al. 2004, the image-quality measure of Sec. 3.1, over volumes [nz][ny][nx]):
 * Gaussian window with sigma 1.5 and 11 taps per axis, normalised; C1 = (0.01 L)^2, C2 = (0.03 L)^2,
 * L = max(gt); mean of the SSIM map over voxels whose window lies inside the volume.  Returns NAN
 * when a dimension is below 11. */
double ora_ssim(const double* gt, const double* pred, int32_t nx, int32_t ny, int32_t nz) {
  const int R = 5;
  if (nx < 2 * R + 1 || ny < 2 * R + 1 || nz < 2 * R + 1) return NAN;
  double w[11], s = 0.0;
  for (int i = -R; i <= R; ++i) s += exp(-(double)(i * i) / (2.0 * 1.5 * 1.5));
  for (int i = -R; i <= R; ++i) w[i + R] = exp(-(double)(i * i) / (2.0 * 1.5 * 1.5)) / s;
  double L = -INFINITY;
  for (int64_t i = 0; i < (int64_t)nx * ny * nz; ++i) if (gt[i] > L) L = gt[i];
  const double c1 = (0.01 * L) * (0.01 * L), c2 = (0.03 * L) * (0.03 * L);
  double total = 0.0;
  int64_t count = 0;
  for (int z = R; z < nz - R; ++z)
    for (int y = R; y < ny - R; ++y)
      for (int x = R; x < nx - R; ++x) {
        double ma = 0.0, mb = 0.0, maa = 0.0, mbb = 0.0, mab = 0.0;
        for (int dz = -R; dz <= R; ++dz)
          for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx) {
              const double ww = w[dz + R] * w[dy + R] * w[dx + R];
              const int64_t i = ((int64_t)(z + dz) * ny + (y + dy)) * nx + (x + dx);
              ma += ww * gt[i];
              mb += ww * pred[i];
              maa += ww * gt[i] * gt[i];
              mbb += ww * pred[i] * pred[i];
              mab += ww * gt[i] * pred[i];
            }
        const double va = maa - ma * ma, vb = mbb - mb * mb, cab = mab - ma * mb;
        total += ((2.0 * ma * mb + c1) * (2.0 * cab + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2));
        ++count;
      }
  return total / (double)count;
}

/* ------------------------------------------------------------------------------------------ */
/* Pre-training for Mapping Consistency Initialization (Sec. 2.1, Sec. 2.4, Eq. 2)             */
/* ------------------------------------------------------------------------------------------ */

/* Trilinear sample of vol[z][y][x] (n^3, voxel-centre convention) at a normalised point:
 * continuous index u = x*n - 1/2 clamped to [0, n-1]; base floor(u) clamped to n-2. */
double ora_trilinear(const float* vol, int32_t n, const float x[3]) {
  int32_t i0[3];
  double f[3];
  for (int k = 0; k < 3; ++k) {
    double u = (double)x[k] * (double)n - 0.5;
    if (u < 0.0) u = 0.0;
    if (u > (double)(n - 1)) u = (double)(n - 1);
    int32_t b = (int32_t)floor(u);
    if (b > n - 2) b = n - 2;
    if (b < 0) b = 0;
    i0[k] = b;
    f[k] = u - (double)b;
  }
  double s = 0.0;
  for (int k = 0; k < 8; ++k) {
    int c0 = k & 1, c1 = (k >> 1) & 1, c2 = (k >> 2) & 1;
    double w = (c0 ? f[0] : 1.0 - f[0]) * (c1 ? f[1] : 1.0 - f[1]) * (c2 ? f[2] : 1.0 - f[2]);
    int64_t xi = i0[0] + c0, yi = i0[1] + c1, zi = i0[2] + c2;
    s += w * (double)vol[(zi * n + yi) * n + xi];
  }
  return s;
}

/* One voxel-loss evaluation over B points for a model with K hash tables (one per pre-training
 * volume) and one shared LayerNorm + MLP.  Parameter layout [K tables][dense block].  Point p uses
 * table tid[p] and target trilinear(vols[tid[p]], xn[p]).  Returns mean |mu - target| and, when
 * grad != NULL, accumulates its gradient (d/dmu = sign(mu - target)/B). */
double ora_voxel_batch(const ora_cfg* c, const double* params, int32_t K, const float* vols, int32_t n,
                       int32_t B, const float* xn, const int32_t* tid, double* mu_out, double* grad) {
  ora_layout o;
  if (make_layout(c, &o)) return NAN;
  int64_t nt = o.n_entries * o.F;
  const double* dn = params + (int64_t)K * nt;
  point_state* st = (point_state*)malloc(sizeof(point_state));
  double loss = 0.0;
  for (int32_t p = 0; p < B; ++p) {
    int32_t k = tid[p];
    point_forward(c, &o, params + (int64_t)k * nt, dn, xn + 3 * (int64_t)p, st);
    double tgt = ora_trilinear(vols + (int64_t)k * n * n * n, n, xn + 3 * (int64_t)p);
    double r = st->mu - tgt;
    if (mu_out) mu_out[p] = st->mu;
    loss += fabs(r);
    if (grad)
      point_backward(c, &o, dn, st, ((r > 0.0) - (r < 0.0)) / (double)B, grad + (int64_t)k * nt,
                     grad + (int64_t)K * nt);
  }
  free(st);
  return loss / (double)B;
}
