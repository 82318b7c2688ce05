// C ABI of libnic (declared in include/nic.h): validation, level table, workspace layout, stream
// handling, and the launch sequence of each entry point.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "nic.h"
#include "nic_device.h"
#include "nic_internal.h"

using namespace nic;

// Scratch of nic_psnr_noalloc, a file-scope device array (each device holds its own copy until the
// process ends): block b of the squared-error kernel writes its (sum, max) pair at [2b, 2b + 1].
// In host code the array's name is not a device address: host code uses only the address that
// hipGetSymbolAddress returned for the current device (scratch_address below).
constexpr int kNoAllocBlocks = 4096;
static __device__ __align__(256) double scratch[2 * kNoAllocBlocks];

namespace {

thread_local std::string g_err;

nic_status fail(nic_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define NIC_HIP(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(NIC_EHIP, "%s: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

constexpr int64_t kAlign = 256;
constexpr int kMaxBwdBlocks = 2048;
constexpr int kMaxReduceBlocks = 512 * 1024 / kReduceThreads;   // bin reduction grid (2 blocks of 1024 threads per CU on 256 CUs)
constexpr int kLossHist = 4096;
constexpr int kSqerrBlocks = 1024;

// Blob of the LayerNorm + MLP weights (Mapping Consistency Initialization transfer): this header,
// then the dense block in the parameter-vector order (FP32).
struct MlpBlobHeader {
  char magic[4];
  uint32_t version;
  int32_t channels, width, depth, out_act, layernorm, n_dense;
  double mu_max, ln_eps;
};
constexpr uint32_t kBlobVersion = 1;

// Training-state blob: this header, then params, adam_m, adam_v (FP32, n_params_padded each).
struct StateHeader {
  char magic[4];
  uint32_t version;
  int32_t cfg_ints[13];   // levels, feats, log2_table, base_res, max_res, depth, width, out_act,
                          // samples, rays, layernorm, precision, n_tables
  int32_t pad_;
  uint64_t seed;
  int64_t n_params_pad;
  int64_t step;
};
constexpr uint32_t kStateVersion = 1;
constexpr int kKinds = 7;   // timed kernel kinds: rays, forward, backward, encode, adam, bin scan, bin reduce

int64_t up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Everything derived from a configuration on the host.
struct Plan {
  LevelTab lt{};
  int32_t res[kMaxLevels]{}, dense[kMaxLevels]{};
  int64_t off[kMaxLevels]{};
  int64_t n_entries = 0, n_table = 0, n_dense = 0, nd_pad = 0, dense_off = 0, n_params_pad = 0;
  int32_t n_tables = 1;
  int64_t o_sqerr = 0;
  int C = 0;
  KernelSet ks;
  // workspace offsets (bytes)
  int64_t o_params, o_grads, o_m, o_v, o_th, o_part, o_rays, o_wsum, o_enc, o_apred, o_absres, o_loss, o_pix;
  int64_t o_counts, o_offs, o_recmax, o_flags, o_mask, o_recs, o_totals, o_binstart, o_bfb, o_bstart, o_split;
  int64_t o_edge = 0, o_ebeg = 0, o_esrc = 0;
  int n_bins = 0;
  // Level-major encoder (k_enc): for bin b, the edge rows edge_src[edge_beg[b] .. edge_beg[b + 1])
  // whose sum is its per-block count (2l: level l's first bin, 2l + 1: its last when that differs);
  // none for a bin strictly inside one level.  enc_lds: bytes of the largest level's histogram.
  std::vector<int32_t> edge_beg, edge_src;
  size_t enc_lds = 0;
  int64_t rec_cap = 0;   // records the record buffer holds
  int64_t bytes = 0;
};

std::string check_config(const nic_config* c) {
  if (!c) return "config is NULL";
  if (c->n_levels != 8 && c->n_levels != 16) return "n_levels must be 8 or 16";
  if (c->feats_per_level != 2) return "feats_per_level must be 2";
  if (c->log2_table < 4 || c->log2_table > 26) return "log2_table must be in [4, 26]";
  if (c->base_res < 1 || c->max_res < c->base_res || c->max_res > 32768) return "need 1 <= base_res <= max_res <= 32768";
  if (c->mlp_width != 32 && c->mlp_width != 64) return "mlp_width must be 32 or 64";
  if (c->mlp_depth < 1 || c->mlp_depth > 4) return "mlp_depth must be in [1, 4]";
  if (c->out_act < 0 || c->out_act > 2) return "out_act must be 0, 1 or 2";
  if (c->samples_per_ray < 32 || c->samples_per_ray > 1024 || c->samples_per_ray % 32)
    return "samples_per_ray must be a multiple of 32 in [32, 1024]";
  if (c->rays_per_step < 1 || c->rays_per_step > 65536) return "rays_per_step must be in [1, 65536]";
  if (c->layernorm != 0 && c->layernorm != 1) return "layernorm must be 0 or 1";
  if (c->precision != 0 && c->precision != 1) return "precision must be 0 or 1";
  if (!(c->mu_max > 0) || !std::isfinite(c->mu_max)) return "mu_max must be positive";
  if (!(c->ln_eps > 0) || !std::isfinite(c->ln_eps)) return "ln_eps must be positive";
  if (!(c->lr > 0) || !std::isfinite(c->lr)) return "lr must be positive";
  if (!(c->beta1 >= 0 && c->beta1 < 1) || !(c->beta2 >= 0 && c->beta2 < 1)) return "betas must be in [0, 1)";
  if (!(c->adam_eps > 0) || !std::isfinite(c->adam_eps)) return "adam_eps must be positive";
  if (c->n_tables < 0 || c->n_tables > 256) return "n_tables must be in [0, 256]";
  return "";
}

std::string check_geometry(const nic_geometry* g, int64_t rays) {
  if (!g) return "geometry is NULL";
  if (!(g->dso > 0) || !(g->dsd > g->dso) || !std::isfinite(g->dsd)) return "need 0 < dso < dsd";
  if (g->det_nu < 1 || g->det_nv < 1) return "detector size must be positive";
  if ((int64_t)g->det_nu * g->det_nv > (1ll << 30)) return "detector too large";
  if (!(g->det_du > 0) || !(g->det_dv > 0)) return "pixel pitch must be positive";
  if (!std::isfinite(g->det_off_u) || !std::isfinite(g->det_off_v)) return "detector offset must be finite";
  for (int k = 0; k < 3; ++k)
    if (!(g->vol_size[k] > 0) || !std::isfinite(g->vol_size[k])) return "vol_size must be positive";
  const double half_diag = 0.5 * std::sqrt(g->vol_size[0] * g->vol_size[0] + g->vol_size[1] * g->vol_size[1]);
  if (!(g->dso > half_diag)) return "source must lie outside the reconstruction box";
  if (g->n_views < 1 || !g->angles_rad) return "need n_views >= 1 and angles";
  for (int v = 0; v < g->n_views; ++v)
    if (!std::isfinite(g->angles_rad[v])) return "angles must be finite";
  if (rays > (int64_t)g->det_nu * g->det_nv) return "rays_per_step exceeds the number of pixels";
  return "";
}

// Level resolutions of the multiresolution grid: N_l = floor(N_min * b^l),
// b = exp((ln N_max - ln N_min)/(L - 1)); a level is dense when (N_l + 1)^3 <= T.
bool make_plan(const nic_config* c, const nic_geometry* g, Plan& p, std::string& err) {
  err = check_config(c);
  if (err.empty() && g) err = check_geometry(g, c->rays_per_step);
  if (!err.empty()) return false;
  const int L = c->n_levels;
  const double b = (L > 1) ? std::exp((std::log((double)c->max_res) - std::log((double)c->base_res)) / (double)(L - 1)) : 1.0;
  const uint64_t T = 1ull << c->log2_table;
  int64_t off = 0;
  for (int l = 0; l < L; ++l) {
    const int32_t N = (int32_t)std::floor((double)c->base_res * std::pow(b, (double)l));
    const double nv = ((double)N + 1.0) * ((double)N + 1.0) * ((double)N + 1.0);
    const bool dense = nv <= (double)T;
    const int64_t size = dense ? (int64_t)nv : (int64_t)T;
    p.res[l] = N;
    p.dense[l] = dense;
    p.off[l] = off;
    p.lt.res[l] = N;
    p.lt.off[l] = (uint32_t)off;
    p.lt.stride[l] = dense ? (uint32_t)(N + 1) : 0u;
    off += size;
  }
  p.lt.mask = (uint32_t)(T - 1);
  p.lt.L = L;
  p.lt.on = 0xFFFFFFFFu;
  p.n_tables = c->n_tables > 1 ? c->n_tables : 1;
  p.n_entries = off;
  p.n_table = off * 2 * p.n_tables;
  if (p.n_table >= (1ll << 31)) { err = "hash tables too large"; return false; }
  p.C = 2 * L;
  p.ks = kernel_set(L, c->mlp_width, c->mlp_depth, c->precision);
  if (!p.ks.valid) { err = "unsupported (levels, width, depth, precision) combination"; return false; }
  p.n_dense = p.ks.n_dense;
  p.nd_pad = p.ks.nd_pad;
  p.dense_off = up(p.n_table, 64);
  p.n_params_pad = up(p.dense_off + p.n_dense, 64);
  // workspace
  const int64_t R = c->rays_per_step, N = c->samples_per_ray;
  int64_t o = 0;
  auto take = [&](int64_t bytes) { const int64_t at = o; o = up(o + bytes, kAlign); return at; };
  p.o_params = take(p.n_params_pad * 4);
  p.o_grads = take(p.n_params_pad * 4);
  p.o_m = take(p.n_params_pad * 4);
  p.o_v = take(p.n_params_pad * 4);
  p.o_th = take(c->precision ? p.n_table * 2 : 0);
  p.o_part = take((int64_t)kMaxBwdBlocks * p.nd_pad * 4);
  p.o_rays = take(R * (int64_t)sizeof(RayRec));
  p.o_wsum = take(R * N / kPtsPerWave * 4);
  p.o_enc = take(R * N * p.C * 4);
  p.o_apred = take(R * 4);
  p.o_absres = take(R * 4);
  p.o_loss = take(kLossHist * 4);
  p.o_pix = take(R * 4);
  // Widest bins that keep the per-bin histogram (k_fwd) and cursors (k_bwd) in LDS beside their tiles.
  {
    const int64_t ent = p.n_entries * p.n_tables;
    const int64_t room = (int64_t)kLdsBytes - (int64_t)std::max(p.ks.fwd_lds, p.ks.bwd_lds);
    int sh = kBinBits;
    while (sh < 31 && ((ent + (1ll << sh) - 1) >> sh) * 4 > room) ++sh;
    if (room <= 0 || ((ent + (1ll << sh) - 1) >> sh) * 4 > room) { err = "gradient bins do not fit in LDS"; return false; }
    p.lt.bin_shift = sh;
    p.n_bins = (int)((ent + (1ll << sh) - 1) >> sh);
  }
  {
    const int sh = p.lt.bin_shift;
    std::vector<std::vector<int32_t>> src(p.n_bins);
    int64_t nbl_max = 1;
    for (int l = 0; l < L; ++l) {
      const int64_t st = p.lt.stride[l];
      const int64_t size = st ? st * st * st : (int64_t)T;
      const int64_t b0 = (int64_t)p.lt.off[l] >> sh, b1 = ((int64_t)p.lt.off[l] + size - 1) >> sh;
      src[b0].push_back(2 * l);
      if (b1 != b0) src[b1].push_back(2 * l + 1);
      nbl_max = std::max(nbl_max, b1 - b0 + 1);
    }
    p.edge_beg.assign(p.n_bins + 1, 0);
    p.edge_src.clear();
    for (int b2 = 0; b2 < p.n_bins; ++b2) {
      p.edge_beg[b2] = (int32_t)p.edge_src.size();
      for (int32_t v : src[b2]) p.edge_src.push_back(v);
    }
    p.edge_beg[p.n_bins] = (int32_t)p.edge_src.size();
    p.enc_lds = (size_t)nbl_max * 4;
    if (p.enc_lds > (size_t)kLdsBytes) { err = "level histogram does not fit in LDS"; return false; }
  }
  const int64_t max_recs = R * N * L * 8;
  if (max_recs >= (1ll << 31)) { err = "too many gradient records per step (rays x samples x levels x 8 >= 2^31)"; return false; }
  p.rec_cap = max_recs;
  const int64_t n_sub = 1ll << (p.lt.bin_shift - kBinBits);
  p.o_totals = take((int64_t)p.n_bins * 4);
  p.o_binstart = take((int64_t)(p.n_bins + 1) * 4);
  p.o_bfb = take((int64_t)kMaxReduceBlocks * 4);
  p.o_bstart = take((int64_t)(kMaxReduceBlocks + 1) * 4);
  p.o_counts = take((int64_t)p.n_bins * kMaxBwdBlocks * 4);
  p.o_offs = take((int64_t)p.n_bins * kMaxBwdBlocks * 4);
  p.o_edge = take(2ll * L * kMaxBwdBlocks * 4);
  p.o_ebeg = take((int64_t)(p.n_bins + 1) * 4);
  p.o_esrc = take((int64_t)std::max<size_t>(1, p.edge_src.size()) * 4);
  p.o_recmax = take(4);
  p.o_flags = take(2 * 4);   // [0] 1 + first step that met a non-finite value (0: none), [1] scratch count
  p.o_mask = take(32 * 4);
  p.o_recs = take(max_recs * (int64_t)sizeof(BinRec));
  p.o_split = take(2ll * kMaxReduceBlocks * n_sub * (2ll << kBinBits) * 8);
  p.o_sqerr = take(2 * kSqerrBlocks * 8);
  p.bytes = o;
  return true;
}

}  // namespace

struct nic_model {
  nic_config cfg;
  Plan plan;
  Geo geo;
  int32_t n_views = 0;
  std::vector<double> ca, sa;
  int32_t h_bits = 1;
  uint32_t n_pix = 0;
  hipStream_t stream = nullptr;
  int n_cu = 0;
  int bwd_grid = 0;
  char* ws = nullptr;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  __half* th = nullptr;
  float *partials = nullptr, *wsum = nullptr, *enc = nullptr, *apred = nullptr, *absres = nullptr, *loss = nullptr;
  RayRec* rays = nullptr;
  int32_t* pix = nullptr;
  uint32_t *counts = nullptr, *offs = nullptr, *totals = nullptr, *bin_start = nullptr;
  int32_t* block_first_bin = nullptr;
  uint32_t* block_start = nullptr;   // [reduce grid + 1] record ranges of the bin reduction
  uint32_t* rec_max = nullptr;
  uint32_t* bad_step = nullptr;   // device: 0, or 1 + the first step whose values were not finite
  uint32_t* count = nullptr;      // device scratch counter
  BinRec* recs = nullptr;
  unsigned long long* split_acc = nullptr;
  int reduce_grid = 0;
  double* sqerr = nullptr;
  const float* vols = nullptr;
  int32_t vol_n = 0;
  const float* proj = nullptr;
  int64_t step = 0;
  int64_t epoch_cached = -1;
  bool grads_dirty = false;   // gradients accumulated by nic_backward and not yet consumed by Adam
  bool masked = false;        // channel mask set by nic_set_channel_mask
  float mask[32] = {};        // host copy (source of the device copy)
  float* mask_dev = nullptr;
  std::vector<int32_t> epoch_order;
  // kernel timing (benchmarks)
  bool timing = false;
  int32_t enc_placement = NIC_ENCODER_AUTO;   // where ray training steps on one table encode
  bool level_major_pays = false;              // the auto rule for this model on this device
  const RaysArgs* next_rays = nullptr;        // set by nic_train: the next step's rays, drawn by this
                                              // step's k_bin_combine
  int64_t rec_cap = 0;        // capacity of recs (records)
  uint32_t* edge = nullptr;
  int32_t *ebeg = nullptr, *esrc = nullptr;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double ms[kKinds] = {};
  int64_t calls[kKinds] = {};
};

namespace {

hipEvent_t ev_get(nic_model* m) {
  if (!m->ev_free.empty()) {
    hipEvent_t e = m->ev_free.back();
    m->ev_free.pop_back();
    return e;
  }
  // timing only (read after the stream has drained): no system-scope fence at each record, which
  // would write back and invalidate the caches between the kernels it brackets
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when timing is on.
struct KTimer {
  nic_model* m;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  KTimer(nic_model* m_, int kind_) : m(m_), kind(kind_) {
    if (m->timing) {
      a = ev_get(m);
      b = ev_get(m);
      if (a) (void)hipEventRecord(a, m->stream);
    }
  }
  ~KTimer() {
    if (m->timing && a && b) {
      (void)hipEventRecord(b, m->stream);
      m->ev_pending.push_back({kind, {a, b}});
    }
  }
};

FwdArgs fwd_args(nic_model* m, int mode, int64_t n_points) {
  FwdArgs a{};
  a.mode = mode;
  a.N = m->cfg.samples_per_ray;
  a.n_points = n_points;
  a.table = m->th ? (const void*)m->th : (const void*)m->params;
  a.dense = m->params + m->plan.dense_off;
  a.lt = m->plan.lt;
  a.geo = m->geo;
  a.rays = m->rays;
  a.seed = m->cfg.seed;
  a.step = (uint32_t)m->step;
  a.layernorm = m->cfg.layernorm;
  a.out_act = m->cfg.out_act;
  a.mu_max = (float)m->cfg.mu_max;
  a.ln_eps = (float)m->cfg.ln_eps;
  a.mask = m->masked ? m->mask_dev : nullptr;
  if (m->masked)
    for (int l = 0; l < a.lt.L; ++l)
      if (m->mask[2 * l] == 0.0f && m->mask[2 * l + 1] == 0.0f) a.lt.on &= ~(1u << l);
  return a;
}

RaysArgs rays_args(const nic_model* m, int32_t view, const int32_t* pix_in, int32_t n_rays, uint32_t step,
                   int32_t* pix_out, float* jitter_out) {
  RaysArgs r{};
  r.geo = m->geo;
  r.ca = m->ca[view];
  r.sa = m->sa[view];
  r.view = view;
  r.N = m->cfg.samples_per_ray;
  r.n_rays = n_rays;
  r.h_bits = m->h_bits;
  r.n_pix = m->n_pix;
  r.step = step;
  r.seed = m->cfg.seed;
  r.pix_in = pix_in;
  r.proj = m->proj;
  r.rays = m->rays;
  r.pix_out = pix_out;
  r.jitter_out = jitter_out;
  return r;
}

nic_status rays(nic_model* m, int32_t view, const int32_t* pix_in, int32_t n_rays, uint32_t step, int32_t* pix_out,
                float* jitter_out) {
  const RaysArgs r = rays_args(m, view, pix_in, n_rays, step, pix_out, jitter_out);
  KTimer kt(m, 0);
  NIC_HIP(launch_rays(r, m->stream));
  return NIC_OK;
}

AdamArgs adam_args(const nic_model* m) {
  const int64_t t = m->step + 1;
  const double bc1 = 1.0 - std::pow(m->cfg.beta1, (double)t);
  const double bc2 = 1.0 - std::pow(m->cfg.beta2, (double)t);
  return AdamArgs{(float)m->cfg.lr, (float)m->cfg.beta1, (float)m->cfg.beta2, (float)m->cfg.adam_eps,
                  (float)(1.0 / bc1), (float)(1.0 / bc2)};
}

nic_status adam(nic_model* m) {
  const int64_t t = m->step + 1;
  const double bc1 = 1.0 - std::pow(m->cfg.beta1, (double)t);
  const double bc2 = 1.0 - std::pow(m->cfg.beta2, (double)t);
  m->grads_dirty = false;
  KTimer kt(m, 4);
  NIC_HIP(launch_adam(m->params, m->grads, m->m, m->v, m->plan.n_params_pad, (float)m->cfg.lr, (float)m->cfg.beta1,
                      (float)m->cfg.beta2, (float)m->cfg.adam_eps, (float)(1.0 / bc1), (float)(1.0 / bc2), m->th,
                      m->plan.n_table, m->bad_step, m->n_cu, m->stream));
  m->step = t;
  return NIC_OK;
}

// Forward + backward (+ reduces) over the points of `a` (rays or voxel-loss mode).  The forward pass
// counts the table-gradient records per (bin, block); the scan turns the counts into write
// offsets; the backward pass writes its records there; the bin reduction sums them into the table
// gradient.  loss_src/loss_n/loss_scale: the per-ray (or per-wave) absolute residuals whose scaled
// sum is the loss written to loss_dev (when not NULL).  fused: the step's Adam update runs inside
// the reductions (table in k_bin_reduce / k_bin_combine, LN + MLP in the dense blocks of
// k_bin_combine) instead of a separate pass over stored gradients; only valid when the gradients
// start at zero.
nic_status fwd_bwd(nic_model* m, FwdArgs a, BwdArgs b, const float* loss_src, int32_t loss_n, float loss_scale,
                   float* loss_dev, bool fused) {
  const Plan& pl = m->plan;
  const int64_t P = a.n_points;
  const int64_t chunks = (P + kPtsPerBlock - 1) / kPtsPerBlock;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(chunks, m->bwd_grid));
  const size_t bin_lds = (size_t)pl.n_bins * 4;
  // Rays on one table: the level-major encoder k_enc computes the encoding and the record counts,
  // and k_fwd only reads the encoding.  Otherwise k_fwd gathers and counts itself.
  const bool want = m->enc_placement == NIC_ENCODER_LEVEL_MAJOR ||
                    (m->enc_placement == NIC_ENCODER_AUTO && m->level_major_pays);
  const bool lvl = want && a.mode == kModeRays && pl.n_tables == 1 && !a.feats && pl.ks.enc;
  a.enc_out = m->enc;
  a.wave_sum = m->wsum;
  a.bin_counts = m->counts;
  a.n_bins = pl.n_bins;
  if (lvl) {
    a.enc_grid = grid;
    a.edge_counts = m->edge;
    {
      KTimer kt(m, 3);
      NIC_HIP(launch_enc(pl.ks, a, pl.enc_lds, m->stream));
    }
    FwdArgs f = a;
    f.enc_pre = m->enc;
    f.enc_out = nullptr;
    f.bin_counts = nullptr;
    f.scan_counts = m->counts;   // k_fwd also runs the offsets' row scans of k_enc's counts
    f.scan_rel = m->offs;
    f.scan_totals = m->totals;
    f.edge_beg = m->ebeg;
    f.edge_src = m->esrc;
    KTimer kt(m, 1);
    NIC_HIP(launch_fwd(pl.ks, f, grid, 0, m->stream));
  } else {
    KTimer kt(m, 1);
    NIC_HIP(launch_fwd(pl.ks, a, grid, bin_lds, m->stream));
  }
  {
    KTimer kt(m, 5);
    NIC_HIP(launch_bin_scan(m->counts, pl.n_bins, grid, m->offs, m->totals, m->bin_start, m->block_start,
                            m->block_first_bin, m->reduce_grid, m->rec_max, lvl ? m->edge : nullptr, m->ebeg,
                            m->esrc, lvl, m->stream));
  }
  b.enc_in = m->enc;
  b.a_pred_out = m->apred;
  b.absres_out = m->absres;
  b.partials = m->partials;
  b.bin_offsets = m->offs;
  b.bin_start = m->bin_start;
  b.recs = m->recs;
  b.rec_cap = (uint32_t)m->rec_cap;
  b.rec_max_bits = m->rec_max;
  b.bad_step = m->bad_step;
  {
    KTimer kt(m, 2);
    NIC_HIP(launch_bwd(pl.ks, a, b, grid, bin_lds, m->stream));
  }
  {
    KTimer kt(m, 6);
    BinReduceArgs br{};
    br.recs = m->recs;
    br.bin_start = m->bin_start;
    br.block_first_bin = m->block_first_bin;
    br.block_start = m->block_start;
    br.n_bins = pl.n_bins;
    br.rec_max_bits = m->rec_max;
    br.grad_table = m->grads;
    br.n_entries = pl.n_entries * pl.n_tables;
    br.bin_shift = pl.lt.bin_shift;
    br.n_sub = 1 << (pl.lt.bin_shift - kBinBits);
    br.split_acc = m->split_acc;
    br.fused = fused ? 1 : 0;
    br.adam = adam_args(m);
    br.p = m->params;
    br.m = m->m;
    br.v = m->v;
    br.th = m->th;
    br.bad_step = m->bad_step;
    DenseReduceArgs& d = br.dense;
    d.partials = m->partials;
    d.n_blocks = grid;
    d.nd_pad = pl.nd_pad;
    d.nd = (int32_t)pl.n_dense;
    d.grad_dense = m->grads + pl.dense_off;
    d.absres = loss_src;
    d.n_rays = loss_n;
    d.inv_R = loss_scale;
    d.loss_out = loss_dev;
    d.fused = fused ? 1 : 0;
    d.adam = br.adam;
    d.p = m->params + pl.dense_off;
    d.m = m->m + pl.dense_off;
    d.v = m->v + pl.dense_off;
    d.bad_step = m->bad_step;
    br.dense_blocks = (d.nd + 63) / 64;
    if (m->next_rays) {
      br.next_rays = *m->next_rays;
      br.ray_blocks = (br.next_rays.n_rays + 1023) / 1024;
    }
    NIC_HIP(launch_bin_reduce(br, m->reduce_grid, m->stream));
  }
  if (fused) m->step += 1;
  else m->grads_dirty = true;
  return NIC_OK;
}

// Ray training pass over the rays currently in m->rays (dA == NULL: L1 loss of Eq. 3).
nic_status ray_fwd_bwd(nic_model* m, int32_t n_rays, const float* jitter, const float* dA, float* loss_dev,
                       bool fused) {
  FwdArgs a = fwd_args(m, kModeRays, (int64_t)n_rays * m->cfg.samples_per_ray);
  a.jitter = jitter;
  BwdArgs b{};
  b.dA_in = dA;
  b.inv_R = 1.0f / (float)n_rays;
  return fwd_bwd(m, a, b, m->absres, n_rays, 1.0f / (float)n_rays, dA ? nullptr : loss_dev, fused);
}

// Voxel-loss pass (Eq. 2) over n_points points.
nic_status voxel_fwd_bwd(nic_model* m, const float* xn, int32_t n_points, float* loss_dev, bool fused) {
  FwdArgs a = fwd_args(m, kModeVoxelLoss, n_points);
  a.xn = xn;
  a.pts_per_table = n_points / m->plan.n_tables;
  a.table_stride = (uint32_t)m->plan.n_entries;
  a.vols = m->vols;
  a.vol_n = m->vol_n;
  BwdArgs b{};
  b.inv_R = 1.0f / (float)n_points;
  b.wave_loss = m->wsum;
  return fwd_bwd(m, a, b, m->wsum, n_points / kPtsPerWave, 1.0f / (float)n_points, loss_dev, fused);
}

// One training step over prepared rays: fused Adam when no gradients are pending, else the
// gradients of this pass are added to the pending ones and a separate Adam pass consumes them.
nic_status ray_train_step(nic_model* m, int32_t n_rays, const float* jitter, float* loss_dev) {
  if (!m->grads_dirty) return ray_fwd_bwd(m, n_rays, jitter, nullptr, loss_dev, true);
  nic_status st = ray_fwd_bwd(m, n_rays, jitter, nullptr, loss_dev, false);
  return st ? st : adam(m);
}

nic_status voxel_train_step(nic_model* m, const float* xn, int32_t n_points, float* loss_dev) {
  if (!m->grads_dirty) return voxel_fwd_bwd(m, xn, n_points, loss_dev, true);
  nic_status st = voxel_fwd_bwd(m, xn, n_points, loss_dev, false);
  return st ? st : adam(m);
}

bool model_ok(const nic_model* m) { return m != nullptr && m->ws != nullptr; }

// After the stream has drained: when a training call met a non-finite value (the device skipped
// that step's update and every later one), rolls the step counter back to that step, clears the
// flag and returns NIC_ENONFINITE.
nic_status take_nonfinite(nic_model* m) {
  uint32_t f = 0;
  NIC_HIP(hipMemcpyAsync(&f, m->bad_step, 4, hipMemcpyDeviceToHost, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  if (f == 0) return NIC_OK;
  // the device holds the low 32 bits of the step index; the first skipped step is the latest step
  // index <= the counter with those bits
  const uint32_t lo = f - 1u;
  const int64_t first = m->step - (int64_t)(uint32_t)((uint32_t)m->step - lo);
  NIC_HIP(launch_fill(reinterpret_cast<float*>(m->bad_step), 1, 0.0f, m->n_cu, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  const int64_t skipped = m->step - first;
  m->step = first;
  return fail(NIC_ENONFINITE,
              "step %lld met a non-finite value (loss, residual, upstream gradient or gradient); it and the %lld "
              "step(s) after it were not applied, the step counter is back at %lld",
              (long long)first, (long long)(skipped > 0 ? skipped - 1 : 0), (long long)first);
}



// nic_psnr_noalloc: one squared-error block per kNoAllocPerBlock voxels, at most kNoAllocBlocks.
constexpr int64_t kNoAllocPerBlock = 65536;   // voxels per block (256 threads x 256)

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices];

// Device address of `scratch` on the current device, looked up once per device.
nic_status scratch_address(double** out) {
  int dev = -1;
  NIC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NIC_EINVAL, "device %d outside [0, %d)", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    NIC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(NIC_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return NIC_OK;
}

}  // namespace

extern "C" {

const char* nic_last_error(void) { return g_err.c_str(); }

nic_status nic_describe(const nic_config* cfg, nic_layout* out) {
  if (!out) return fail(NIC_EINVAL, "out is NULL");
  Plan p;
  std::string err;
  if (!make_plan(cfg, nullptr, p, err)) return fail(NIC_EINVAL, "%s", err.c_str());
  memset(out, 0, sizeof *out);
  out->n_levels = cfg->n_levels;
  for (int l = 0; l < cfg->n_levels; ++l) {
    out->res[l] = p.res[l];
    out->dense[l] = p.dense[l];
    out->offset[l] = p.off[l];
  }
  out->n_entries = p.n_entries;
  out->n_table = p.n_table;
  out->n_dense = p.n_dense;
  out->dense_offset = p.dense_off;
  out->n_params_padded = p.n_params_pad;
  out->bin_shift = p.lt.bin_shift;
  out->n_bins = p.n_bins;
  return NIC_OK;
}

size_t nic_workspace_size(const nic_config* cfg, const nic_geometry* geom) {
  Plan p;
  std::string err;
  if (!geom || !make_plan(cfg, geom, p, err)) {
    g_err = geom ? err : "geometry is NULL";
    return 0;
  }
  return (size_t)p.bytes;
}

nic_status nic_create(const nic_config* cfg, const nic_geometry* geom, void* hip_stream, void* workspace,
                      size_t ws_bytes, nic_model** out) {
  if (!out) return fail(NIC_EINVAL, "out is NULL");
  *out = nullptr;
  Plan p;
  std::string err;
  if (!geom) return fail(NIC_EINVAL, "geometry is NULL");
  if (!make_plan(cfg, geom, p, err)) return fail(NIC_EINVAL, "%s", err.c_str());
  if (!workspace) return fail(NIC_EINVAL, "workspace is NULL");
  if (((uintptr_t)workspace) % kAlign) return fail(NIC_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < (size_t)p.bytes) return fail(NIC_ENOMEM, "workspace has %zu bytes, needs %lld", ws_bytes, (long long)p.bytes);

  nic_model* m = new nic_model();
  m->cfg = *cfg;
  m->plan = p;
  m->stream = (hipStream_t)hip_stream;
  m->n_views = geom->n_views;
  m->ca.resize(geom->n_views);
  m->sa.resize(geom->n_views);
  for (int v = 0; v < geom->n_views; ++v) {
    m->ca[v] = std::cos(geom->angles_rad[v]);
    m->sa[v] = std::sin(geom->angles_rad[v]);
  }
  Geo& g = m->geo;
  g.dso = geom->dso;
  g.back = geom->dsd - geom->dso;
  g.du = geom->det_du;
  g.dv = geom->det_dv;
  g.off_u = geom->det_off_u;
  g.off_v = geom->det_off_v;
  for (int k = 0; k < 3; ++k) {
    g.vol[k] = geom->vol_size[k];
    g.inv_vol[k] = 1.0 / geom->vol_size[k];
  }
  g.nu = geom->det_nu;
  g.nv = geom->det_nv;
  m->n_pix = (uint32_t)((int64_t)geom->det_nu * geom->det_nv);
  int bits = 0;
  while ((1ll << bits) < (int64_t)m->n_pix) ++bits;
  if (bits & 1) ++bits;
  if (bits < 2) bits = 2;
  m->h_bits = bits / 2;

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&m->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t bin_lds = (size_t)p.n_bins * 4;
  if (e == hipSuccess)
    e = hipFuncSetAttribute(p.ks.fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(p.ks.fwd_lds + bin_lds));
  if (e == hipSuccess)
    e = hipFuncSetAttribute(p.ks.bwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(p.ks.bwd_lds + bin_lds));
  if (e == hipSuccess)
    e = hipFuncSetAttribute(p.ks.enc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.enc_lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(bin_reduce_kernel(true), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bin_reduce_lds());
  if (e == hipSuccess)
    e = hipFuncSetAttribute(bin_reduce_kernel(false), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bin_reduce_lds());
  int per_cu = 0, per_cu_red = 0, l2 = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&l2, hipDeviceAttributeL2CacheSize, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, p.ks.bwd, kBlock, p.ks.bwd_lds + bin_lds);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_red, bin_reduce_kernel(true), kReduceThreads, bin_reduce_lds());
  if (e != hipSuccess) {
    delete m;
    return fail(NIC_EHIP, "device query: %s", hipGetErrorString(e));
  }
  m->bwd_grid = std::max(1, std::min(kMaxBwdBlocks, m->n_cu * std::max(1, per_cu)));
  // The level-major encoder pays when the whole table overflows an XCD's L2 but one level's table
  // fits in about twice that (measured: 2 and 4 MB levels gain 1.3-1.7x on the encode, 8 MB ones
  // 1.1x, 16 MB ones lose; a table that fits in L2 as a whole loses the extra pass).
  {
    const int64_t eb = cfg->precision ? 4 : 8, l2b = l2 > 0 ? l2 : (4 << 20);
    int64_t lvl_max = 0;
    for (int l = 0; l < cfg->n_levels; ++l) {
      const int64_t st = p.lt.stride[l];
      lvl_max = std::max<int64_t>(lvl_max, (st ? st * st * st : (int64_t)p.lt.mask + 1) * eb);
    }
    m->level_major_pays = p.n_entries * eb > l2b && lvl_max <= 2 * l2b;
  }
  m->reduce_grid = std::max(1, std::min(kMaxReduceBlocks, m->n_cu * std::max(1, per_cu_red)));

  char* ws = (char*)workspace;
  m->ws = ws;
  m->params = (float*)(ws + p.o_params);
  m->grads = (float*)(ws + p.o_grads);
  m->m = (float*)(ws + p.o_m);
  m->v = (float*)(ws + p.o_v);
  m->th = cfg->precision ? (__half*)(ws + p.o_th) : nullptr;
  m->partials = (float*)(ws + p.o_part);
  m->rays = (RayRec*)(ws + p.o_rays);
  m->wsum = (float*)(ws + p.o_wsum);
  m->enc = (float*)(ws + p.o_enc);
  m->apred = (float*)(ws + p.o_apred);
  m->absres = (float*)(ws + p.o_absres);
  m->loss = (float*)(ws + p.o_loss);
  m->pix = (int32_t*)(ws + p.o_pix);
  m->counts = (uint32_t*)(ws + p.o_counts);
  m->offs = (uint32_t*)(ws + p.o_offs);
  m->block_first_bin = (int32_t*)(ws + p.o_bfb);
  m->block_start = (uint32_t*)(ws + p.o_bstart);
  m->rec_max = (uint32_t*)(ws + p.o_recmax);
  m->bad_step = (uint32_t*)(ws + p.o_flags);
  m->count = m->bad_step + 1;
  m->mask_dev = (float*)(ws + p.o_mask);
  m->recs = (BinRec*)(ws + p.o_recs);
  m->rec_cap = p.rec_cap;
  m->edge = (uint32_t*)(ws + p.o_edge);
  m->ebeg = (int32_t*)(ws + p.o_ebeg);
  m->esrc = (int32_t*)(ws + p.o_esrc);
  m->split_acc = (unsigned long long*)(ws + p.o_split);
  m->totals = (uint32_t*)(ws + p.o_totals);
  m->bin_start = (uint32_t*)(ws + p.o_binstart);
  m->sqerr = (double*)(ws + p.o_sqerr);
  *out = m;
  nic_status st = NIC_OK;
  if (hipMemcpy(m->ebeg, p.edge_beg.data(), p.edge_beg.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      (!p.edge_src.empty() &&
       hipMemcpy(m->esrc, p.edge_src.data(), p.edge_src.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
    st = fail(NIC_EHIP, "copying the bin tables failed");
  if (st == NIC_OK && launch_fill(reinterpret_cast<float*>(m->bad_step), 2, 0.0f, m->n_cu, m->stream) != hipSuccess)
    st = fail(NIC_EHIP, "clearing the flags failed");
  if (st == NIC_OK) st = nic_init_params(m, cfg->seed);
  if (st != NIC_OK) {
    delete m;
    *out = nullptr;
    return st;
  }
  return NIC_OK;
}

void nic_destroy(nic_model* m) {
  if (!m) return;
  for (auto& pe : m->ev_pending) {
    (void)hipEventDestroy(pe.second.first);
    (void)hipEventDestroy(pe.second.second);
  }
  for (hipEvent_t e : m->ev_free) (void)hipEventDestroy(e);
  delete m;
}

nic_status nic_set_encoder_placement(nic_model* m, int32_t placement) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (placement != NIC_ENCODER_AUTO && placement != NIC_ENCODER_LEVEL_MAJOR && placement != NIC_ENCODER_IN_FORWARD)
    return fail(NIC_EINVAL, "placement must be NIC_ENCODER_AUTO, _LEVEL_MAJOR or _IN_FORWARD");
  m->enc_placement = placement;
  return NIC_OK;
}

int32_t nic_encoder_level_major(const nic_model* m) {
  if (!m) return 0;
  const bool want = m->enc_placement == NIC_ENCODER_LEVEL_MAJOR ||
                    (m->enc_placement == NIC_ENCODER_AUTO && m->level_major_pays);
  return want && m->plan.n_tables == 1 ? 1 : 0;
}

nic_status nic_set_timing(nic_model* m, int32_t enable) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  m->timing = enable != 0;
  for (int k = 0; k < kKinds; ++k) { m->ms[k] = 0; m->calls[k] = 0; }
  return NIC_OK;
}

nic_status nic_kernel_times(nic_model* m, double* ms, int64_t* calls, int32_t* count) {
  if (!model_ok(m) || !ms || !calls || !count) return fail(NIC_EINVAL, "NULL argument");
  NIC_HIP(hipStreamSynchronize(m->stream));
  for (auto& pe : m->ev_pending) {
    float t = 0.0f;
    NIC_HIP(hipEventElapsedTime(&t, pe.second.first, pe.second.second));
    m->ms[pe.first] += t;
    m->calls[pe.first] += 1;
    m->ev_free.push_back(pe.second.first);
    m->ev_free.push_back(pe.second.second);
  }
  m->ev_pending.clear();
  for (int k = 0; k < kKinds; ++k) { ms[k] = m->ms[k]; calls[k] = m->calls[k]; }
  *count = kKinds;
  return NIC_OK;
}

nic_status nic_init_params(nic_model* m, uint64_t seed) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  const Plan& p = m->plan;
  const int C = p.C, W = m->cfg.mlp_width;
  InitArgs ia{};
  ia.seed = seed;
  ia.n_dense = p.n_dense;
  ia.ln_end = 2 * C;
  ia.first_layer_end = 2 * C + (int64_t)W * C + W;
  ia.fan0 = C;
  ia.width = W;
  NIC_HIP(launch_fill(m->params, p.n_params_pad, 0.0f, m->n_cu, m->stream));
  NIC_HIP(launch_fill(m->grads, p.n_params_pad, 0.0f, m->n_cu, m->stream));
  m->grads_dirty = false;
  NIC_HIP(launch_fill(m->m, p.n_params_pad, 0.0f, m->n_cu, m->stream));
  NIC_HIP(launch_fill(m->v, p.n_params_pad, 0.0f, m->n_cu, m->stream));
  NIC_HIP(launch_init(m->params, p.n_table, p.dense_off, ia, m->n_cu, m->stream));
  if (m->th) NIC_HIP(launch_to_half(m->params, m->th, p.n_table, m->n_cu, m->stream));
  m->step = 0;
  return NIC_OK;
}

nic_status nic_set_projections(nic_model* m, const float* proj_dev) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (!proj_dev) return fail(NIC_EINVAL, "projections are NULL");
  const int64_t n = (int64_t)m->n_views * m->n_pix;
  NIC_HIP(launch_count_nonfinite(proj_dev, n, m->count, m->n_cu, m->stream));
  uint32_t bad = 0;
  NIC_HIP(hipMemcpyAsync(&bad, m->count, 4, hipMemcpyDeviceToHost, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  if (bad) return fail(NIC_ENONFINITE, "%u of the %lld projection values are not finite", bad, (long long)n);
  m->proj = proj_dev;
  return NIC_OK;
}

nic_status nic_sync(nic_model* m) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  NIC_HIP(hipStreamSynchronize(m->stream));
  return take_nonfinite(m);
}

nic_status nic_tensors(nic_model* m, nic_tensor* out, int32_t* count) {
  if (!model_ok(m) || !out || !count) return fail(NIC_EINVAL, "NULL argument");
  const int64_t n = m->plan.n_params_pad;
  out[0] = nic_tensor{m->params, n, 0, 0};
  out[1] = nic_tensor{m->grads, n, 0, 0};
  out[2] = nic_tensor{m->m, n, 0, 0};
  out[3] = nic_tensor{m->v, n, 0, 0};
  out[4] = nic_tensor{m->th, m->th ? m->plan.n_table : 0, 1, 0};
  *count = 5;
  return NIC_OK;
}

nic_status nic_sync_params(nic_model* m) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (m->th) NIC_HIP(launch_to_half(m->params, m->th, m->plan.n_table, m->n_cu, m->stream));
  return NIC_OK;
}

int64_t nic_get_step(const nic_model* m) { return m ? m->step : -1; }

int32_t nic_view_for_step(const nic_model* m_, int64_t step) {
  nic_model* m = const_cast<nic_model*>(m_);
  if (!m || step < 0) return -1;
  const int32_t V = m->n_views;
  const int64_t e = step / V;
  if (e != m->epoch_cached) {
    std::vector<std::pair<uint32_t, int32_t>> key(V);
    for (int32_t v = 0; v < V; ++v) key[v] = {philox_w0(m->cfg.seed, (uint32_t)v, (uint32_t)e, 0, kViews), v};
    std::sort(key.begin(), key.end());
    m->epoch_order.resize(V);
    for (int32_t k = 0; k < V; ++k) m->epoch_order[k] = key[k].second;
    m->epoch_cached = e;
  }
  return m->epoch_order[step % V];
}

nic_status nic_draw_rays(nic_model* m, int64_t step, int32_t* pix_dev, float* jitter_dev) {
  if (!model_ok(m) || !pix_dev || !jitter_dev) return fail(NIC_EINVAL, "NULL argument");
  if (step < 0) return fail(NIC_EINVAL, "step must be >= 0");
  return rays(m, 0, nullptr, m->cfg.rays_per_step, (uint32_t)step, pix_dev, jitter_dev);
}

nic_status nic_step(nic_model* m, int32_t view, const int32_t* pix_dev, const float* jitter_dev, float* loss_dev) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (view < 0 || view >= m->n_views) return fail(NIC_EINVAL, "view %d out of range", view);
  if (!m->proj) return fail(NIC_ESTATE, "projections not set");
  const int32_t R = m->cfg.rays_per_step;
  nic_status st = rays(m, view, pix_dev, R, (uint32_t)m->step, nullptr, nullptr);
  if (st) return st;
  return ray_train_step(m, R, jitter_dev, loss_dev ? loss_dev : m->loss);
}

nic_status nic_train(nic_model* m, int32_t n_steps, float* loss_host) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (n_steps < 0) return fail(NIC_EINVAL, "n_steps must be >= 0");
  if (!m->proj) return fail(NIC_ESTATE, "projections not set");
  bool bad = false;
  nic_status st = NIC_OK;
  const int32_t R = m->cfg.rays_per_step;
  bool drawn = false;   // this step's rays were drawn by the previous step's combine kernel
  for (int32_t k0 = 0; k0 < n_steps; k0 += kLossHist) {
    const int32_t kn = std::min<int32_t>(kLossHist, n_steps - k0);
    for (int32_t k = 0; k < kn; ++k) {
      const int64_t t = m->step;
      if (!drawn) {
        st = rays(m, nic_view_for_step(m, t), nullptr, R, (uint32_t)t, nullptr, nullptr);
        if (st) return st;
      }
      // a step that is not the call's last draws the next step's rays (step t + 1) in its combine
      // kernel, once its backward pass no longer reads the ray buffer
      const bool more = k0 + k + 1 < n_steps;
      RaysArgs next{};
      if (more) next = rays_args(m, nic_view_for_step(m, t + 1), nullptr, R, (uint32_t)(t + 1), nullptr, nullptr);
      m->next_rays = more ? &next : nullptr;
      st = ray_train_step(m, R, nullptr, m->loss + k);   // advances m->step to t + 1
      m->next_rays = nullptr;
      if (st) return st;
      drawn = more;
    }
    if (loss_host) {
      NIC_HIP(hipMemcpyAsync(loss_host + k0, m->loss, kn * sizeof(float), hipMemcpyDeviceToHost, m->stream));
      NIC_HIP(hipStreamSynchronize(m->stream));
      for (int32_t k = 0; k < kn; ++k)
        if (!std::isfinite(loss_host[k0 + k])) bad = true;
      st = take_nonfinite(m);
      if (st) return st;
    }
  }
  if (bad) return fail(NIC_ENONFINITE, "non-finite loss");
  return NIC_OK;
}

nic_status nic_forward(nic_model* m, int32_t view, const int32_t* pix_dev, const float* jitter_dev, int32_t n_rays,
                       float* a_pred_dev) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (view < 0 || view >= m->n_views) return fail(NIC_EINVAL, "view %d out of range", view);
  if (n_rays < 0 || n_rays > m->cfg.rays_per_step) return fail(NIC_EINVAL, "n_rays out of range");
  if (n_rays == 0) return NIC_OK;
  if (!pix_dev || !jitter_dev || !a_pred_dev) return fail(NIC_EINVAL, "NULL argument");
  nic_status st = rays(m, view, pix_dev, n_rays, (uint32_t)m->step, nullptr, nullptr);
  if (st) return st;
  const int64_t P = (int64_t)n_rays * m->cfg.samples_per_ray;
  FwdArgs a = fwd_args(m, kModeRays, P);
  a.jitter = jitter_dev;
  a.wave_sum = m->wsum;
  NIC_HIP(launch_fwd(m->plan.ks, a, 0, 0, m->stream));
  NIC_HIP(launch_raysum(m->wsum, m->cfg.samples_per_ray / kPtsPerWave, n_rays, a_pred_dev, m->stream));
  return NIC_OK;
}

nic_status nic_backward(nic_model* m, int32_t view, const int32_t* pix_dev, const float* jitter_dev, int32_t n_rays,
                        const float* dA_dev) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (view < 0 || view >= m->n_views) return fail(NIC_EINVAL, "view %d out of range", view);
  if (n_rays < 0 || n_rays > m->cfg.rays_per_step) return fail(NIC_EINVAL, "n_rays out of range");
  if (n_rays == 0) return NIC_OK;
  if (!pix_dev || !jitter_dev || !dA_dev) return fail(NIC_EINVAL, "NULL argument");
  nic_status st = rays(m, view, pix_dev, n_rays, (uint32_t)m->step, nullptr, nullptr);
  if (st) return st;
  return ray_fwd_bwd(m, n_rays, jitter_dev, dA_dev, nullptr, false);
}

nic_status nic_adam(nic_model* m) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  return adam(m);
}

nic_status nic_zero_grad(nic_model* m) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  NIC_HIP(launch_fill(m->grads, m->plan.n_params_pad, 0.0f, m->n_cu, m->stream));
  m->grads_dirty = false;
  return NIC_OK;
}

nic_status nic_query(nic_model* m, const float* xn_dev, int64_t n, float* mu_dev) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (n < 0) return fail(NIC_EINVAL, "n must be >= 0");
  if (n == 0) return NIC_OK;
  if (!xn_dev || !mu_dev) return fail(NIC_EINVAL, "NULL argument");
  FwdArgs a = fwd_args(m, kModePoints, n);
  a.xn = xn_dev;
  a.mu_out = mu_dev;
  NIC_HIP(launch_fwd(m->plan.ks, a, 0, 0, m->stream));
  return NIC_OK;
}

nic_status nic_field_from_features(nic_model* m, const float* enc_dev, int64_t n, float* mu_dev) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (n < 0) return fail(NIC_EINVAL, "n must be >= 0");
  if (n == 0) return NIC_OK;
  if (!enc_dev || !mu_dev) return fail(NIC_EINVAL, "NULL argument");
  FwdArgs a = fwd_args(m, kModeFeatures, n);
  a.feats = enc_dev;
  a.mu_out = mu_dev;
  NIC_HIP(launch_fwd(m->plan.ks, a, 0, 0, m->stream));
  return NIC_OK;
}

nic_status nic_channel_spectrum(nic_model* m, int32_t g_max, float* hf_host) {
  if (!model_ok(m) || !hf_host) return fail(NIC_EINVAL, "NULL argument");
  if (g_max < 4 || g_max > 64) return fail(NIC_EINVAL, "g_max must be in [4, 64]");
  const Plan& pl = m->plan;
  const int C = pl.C;
  // scratch inside the record buffer (unused between training steps): points, encodings, 2 fields
  const int64_t n_max = (int64_t)g_max * g_max * g_max;
  const int64_t need = n_max * 12 + n_max * C * 4 + 2 * n_max * 16 + 64;
  if (need > pl.o_split - pl.o_recs) return fail(NIC_EINVAL, "record buffer too small for a %d^3 probe", g_max);
  char* base = (char*)m->recs;
  float* xn = (float*)base;
  float* enc = (float*)(base + n_max * 12);
  double2* b0 = (double2*)(base + ((n_max * 12 + n_max * C * 4 + 15) & ~(int64_t)15));
  double2* b1 = b0 + n_max;
  const int nb = kSqerrBlocks;
  std::vector<double> h(2 * (size_t)nb);
  for (int l = 0; l < pl.lt.L; ++l) {
    const int N = pl.lt.res[l];
    const int G = std::min(g_max, N);
    const int v0 = (N - G) / 2;
    NIC_HIP(launch_probe_points(N, v0, G, xn, m->stream));
    NIC_HIP(launch_encode(pl.lt, m->params, 0, xn, (int64_t)G * G * G, enc, nullptr, m->stream));
    for (int f = 0; f < 2; ++f) {
      NIC_HIP(launch_channel_power(enc, C, 2 * l + f, G, b0, b1, m->sqerr, nb, m->stream));
      NIC_HIP(hipMemcpyAsync(h.data(), m->sqerr, h.size() * 8, hipMemcpyDeviceToHost, m->stream));
      NIC_HIP(hipStreamSynchronize(m->stream));
      double hi = 0.0, tot = 0.0;
      for (int b = 0; b < nb; ++b) {
        hi += h[2 * b];
        tot += h[2 * b + 1];
      }
      hf_host[2 * l + f] = tot > 0.0 ? (float)(hi / tot) : 0.0f;
    }
  }
  return NIC_OK;
}

nic_status nic_set_channel_mask(nic_model* m, const float* mask_host, int32_t n) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (!mask_host) {
    m->masked = false;
    return NIC_OK;
  }
  if (n != m->plan.C) return fail(NIC_EINVAL, "mask needs %d channels, got %d", m->plan.C, n);
  for (int c = 0; c < n; ++c) {
    if (!std::isfinite(mask_host[c])) return fail(NIC_EINVAL, "mask value %d is not finite", c);
    m->mask[c] = mask_host[c];
  }
  NIC_HIP(hipMemcpyAsync(m->mask_dev, m->mask, (size_t)n * 4, hipMemcpyHostToDevice, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  m->masked = true;
  return NIC_OK;
}

nic_status nic_render_volume(nic_model* m, const int32_t dims[3], float* vol_dev) {
  if (!model_ok(m) || !dims || !vol_dev) return fail(NIC_EINVAL, "NULL argument");
  for (int k = 0; k < 3; ++k)
    if (dims[k] < 1 || dims[k] > 4096) return fail(NIC_EINVAL, "dims must be in [1, 4096]");
  const int64_t n = (int64_t)dims[0] * dims[1] * dims[2];
  FwdArgs a = fwd_args(m, kModeVoxels, n);
  for (int k = 0; k < 3; ++k) a.dims[k] = dims[k];
  a.mu_out = vol_dev;
  NIC_HIP(launch_fwd(m->plan.ks, a, 0, 0, m->stream));
  return NIC_OK;
}

nic_status nic_encode(nic_model* m, const float* xn_dev, int64_t n, float* enc_dev, uint32_t* idx_dev) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (n < 0) return fail(NIC_EINVAL, "n must be >= 0");
  if (n == 0) return NIC_OK;
  if (!xn_dev || !enc_dev) return fail(NIC_EINVAL, "NULL argument");
  NIC_HIP(launch_encode(m->plan.lt, m->th ? (const void*)m->th : (const void*)m->params, m->th ? 1 : 0, xn_dev, n,
                        enc_dev, idx_dev, m->stream));
  return NIC_OK;
}

nic_status nic_set_volumes(nic_model* m, const float* vols_dev, int32_t n) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (!vols_dev || n < 2 || n > 2048) return fail(NIC_EINVAL, "need volumes and 2 <= n <= 2048");
  m->vols = vols_dev;
  m->vol_n = n;
  return NIC_OK;
}

static nic_status check_voxel_args(nic_model* m, int32_t n_points) {
  const int32_t K = m->plan.n_tables;
  if (!m->vols) return fail(NIC_ESTATE, "target volumes not set");
  if (n_points < 32 * K || n_points % (32 * K))
    return fail(NIC_EINVAL, "n_points must be a positive multiple of 32 * n_tables");
  if ((int64_t)n_points > (int64_t)m->cfg.rays_per_step * m->cfg.samples_per_ray)
    return fail(NIC_EINVAL, "n_points exceeds rays_per_step * samples_per_ray");
  return NIC_OK;
}

nic_status nic_voxel_step(nic_model* m, const float* xn_dev, int32_t n_points, float* loss_dev) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  nic_status st = check_voxel_args(m, n_points);
  if (st) return st;
  return voxel_train_step(m, xn_dev, n_points, loss_dev ? loss_dev : m->loss);
}

nic_status nic_voxel_train(nic_model* m, int32_t n_steps, int32_t n_points, float* loss_host) {
  if (!model_ok(m)) return fail(NIC_EINVAL, "model is NULL");
  if (n_steps < 0) return fail(NIC_EINVAL, "n_steps must be >= 0");
  nic_status st = check_voxel_args(m, n_points);
  if (st) return st;
  bool bad = false;
  for (int32_t k0 = 0; k0 < n_steps; k0 += kLossHist) {
    const int32_t kn = std::min<int32_t>(kLossHist, n_steps - k0);
    for (int32_t k = 0; k < kn; ++k) {
      st = voxel_train_step(m, nullptr, n_points, m->loss + k);
      if (st) return st;
    }
    if (loss_host) {
      NIC_HIP(hipMemcpyAsync(loss_host + k0, m->loss, kn * sizeof(float), hipMemcpyDeviceToHost, m->stream));
      NIC_HIP(hipStreamSynchronize(m->stream));
      for (int32_t k = 0; k < kn; ++k)
        if (!std::isfinite(loss_host[k0 + k])) bad = true;
      st = take_nonfinite(m);
      if (st) return st;
    }
  }
  if (bad) return fail(NIC_ENONFINITE, "non-finite loss");
  return NIC_OK;
}

nic_status nic_export_mlp(nic_model* m, void* buf, size_t* bytes) {
  if (!model_ok(m) || !bytes) return fail(NIC_EINVAL, "NULL argument");
  const size_t need = sizeof(MlpBlobHeader) + (size_t)m->plan.n_dense * sizeof(float);
  if (!buf) {
    *bytes = need;
    return NIC_OK;
  }
  if (*bytes < need) return fail(NIC_EINVAL, "buffer too small (%zu < %zu)", *bytes, need);
  MlpBlobHeader h{};
  memcpy(h.magic, "NICM", 4);
  h.version = kBlobVersion;
  h.channels = m->plan.C;
  h.width = m->cfg.mlp_width;
  h.depth = m->cfg.mlp_depth;
  h.out_act = m->cfg.out_act;
  h.layernorm = m->cfg.layernorm;
  h.n_dense = (int32_t)m->plan.n_dense;
  h.mu_max = m->cfg.mu_max;
  h.ln_eps = m->cfg.ln_eps;
  memcpy(buf, &h, sizeof h);
  NIC_HIP(hipMemcpyAsync((char*)buf + sizeof h, m->params + m->plan.dense_off, (size_t)m->plan.n_dense * 4,
                         hipMemcpyDeviceToHost, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  *bytes = need;
  return NIC_OK;
}

nic_status nic_import_mlp(nic_model* m, const void* buf, size_t bytes) {
  if (!model_ok(m) || !buf) return fail(NIC_EINVAL, "NULL argument");
  if (bytes < sizeof(MlpBlobHeader)) return fail(NIC_EVERSION, "blob too short");
  MlpBlobHeader h;
  memcpy(&h, buf, sizeof h);
  if (memcmp(h.magic, "NICM", 4) || h.version != kBlobVersion) return fail(NIC_EVERSION, "not an MLP blob");
  if (h.channels != m->plan.C || h.width != m->cfg.mlp_width || h.depth != m->cfg.mlp_depth ||
      h.out_act != m->cfg.out_act || h.layernorm != m->cfg.layernorm || h.n_dense != m->plan.n_dense)
    return fail(NIC_EVERSION, "blob of another network shape");
  if (h.mu_max != m->cfg.mu_max || h.ln_eps != m->cfg.ln_eps)
    return fail(NIC_EVERSION, "blob of another output scale or LayerNorm epsilon (mu_max %g, ln_eps %g)", h.mu_max,
                h.ln_eps);
  if (bytes < sizeof h + (size_t)h.n_dense * 4) return fail(NIC_EVERSION, "blob truncated");
  NIC_HIP(hipMemcpyAsync(m->params + m->plan.dense_off, (const char*)buf + sizeof h, (size_t)h.n_dense * 4,
                         hipMemcpyHostToDevice, m->stream));
  NIC_HIP(launch_fill(m->m + m->plan.dense_off, m->plan.n_dense, 0.0f, m->n_cu, m->stream));
  NIC_HIP(launch_fill(m->v + m->plan.dense_off, m->plan.n_dense, 0.0f, m->n_cu, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  return NIC_OK;
}

static void state_header(const nic_model* m, StateHeader& h) {
  memset(&h, 0, sizeof h);
  memcpy(h.magic, "NICS", 4);
  h.version = kStateVersion;
  const nic_config& c = m->cfg;
  const int32_t v[13] = {c.n_levels, c.feats_per_level, c.log2_table, c.base_res, c.max_res, c.mlp_depth,
                         c.mlp_width, c.out_act, c.samples_per_ray, c.rays_per_step, c.layernorm, c.precision,
                         m->plan.n_tables};
  memcpy(h.cfg_ints, v, sizeof v);
  h.seed = c.seed;
  h.n_params_pad = m->plan.n_params_pad;
  h.step = m->step;
}

nic_status nic_save_state(nic_model* m, void* buf, size_t* bytes) {
  if (!model_ok(m) || !bytes) return fail(NIC_EINVAL, "NULL argument");
  const size_t n = (size_t)m->plan.n_params_pad * 4;
  const size_t need = sizeof(StateHeader) + 3 * n;
  if (!buf) {
    *bytes = need;
    return NIC_OK;
  }
  if (*bytes < need) return fail(NIC_EINVAL, "buffer too small (%zu < %zu)", *bytes, need);
  NIC_HIP(hipStreamSynchronize(m->stream));
  nic_status st = take_nonfinite(m);   // the saved step counter must match the parameters
  if (st) return st;
  StateHeader h;
  state_header(m, h);
  memcpy(buf, &h, sizeof h);
  char* dst = (char*)buf + sizeof h;
  NIC_HIP(hipMemcpyAsync(dst, m->params, n, hipMemcpyDeviceToHost, m->stream));
  NIC_HIP(hipMemcpyAsync(dst + n, m->m, n, hipMemcpyDeviceToHost, m->stream));
  NIC_HIP(hipMemcpyAsync(dst + 2 * n, m->v, n, hipMemcpyDeviceToHost, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  *bytes = need;
  return NIC_OK;
}

nic_status nic_load_state(nic_model* m, const void* buf, size_t bytes) {
  if (!model_ok(m) || !buf) return fail(NIC_EINVAL, "NULL argument");
  if (bytes < sizeof(StateHeader)) return fail(NIC_EVERSION, "state blob too short");
  StateHeader h, mine;
  memcpy(&h, buf, sizeof h);
  state_header(m, mine);
  if (memcmp(h.magic, "NICS", 4) || h.version != kStateVersion) return fail(NIC_EVERSION, "not a state blob");
  if (memcmp(h.cfg_ints, mine.cfg_ints, sizeof h.cfg_ints) || h.seed != mine.seed ||
      h.n_params_pad != mine.n_params_pad)
    return fail(NIC_EVERSION, "state of another configuration");
  const size_t n = (size_t)m->plan.n_params_pad * 4;
  if (bytes < sizeof h + 3 * n) return fail(NIC_EVERSION, "state blob truncated");
  const char* src = (const char*)buf + sizeof h;
  NIC_HIP(hipMemcpyAsync(m->params, src, n, hipMemcpyHostToDevice, m->stream));
  NIC_HIP(hipMemcpyAsync(m->m, src + n, n, hipMemcpyHostToDevice, m->stream));
  NIC_HIP(hipMemcpyAsync(m->v, src + 2 * n, n, hipMemcpyHostToDevice, m->stream));
  NIC_HIP(launch_fill(m->grads, m->plan.n_params_pad, 0.0f, m->n_cu, m->stream));
  m->grads_dirty = false;
  if (m->th) NIC_HIP(launch_to_half(m->params, m->th, m->plan.n_table, m->n_cu, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  m->step = h.step;
  return NIC_OK;
}

nic_status nic_psnr(nic_model* m, const float* gt_dev, const float* pred_dev, int64_t n, double* psnr_host) {
  if (!model_ok(m) || !gt_dev || !pred_dev || !psnr_host) return fail(NIC_EINVAL, "NULL argument");
  if (n < 1) return fail(NIC_EINVAL, "n must be >= 1");
  const int nb = (int)std::min<int64_t>(kSqerrBlocks, (n + 255) / 256);
  NIC_HIP(launch_sqerr(gt_dev, pred_dev, n, m->sqerr, nb, m->stream));
  std::vector<double> h(2 * (size_t)nb);
  NIC_HIP(hipMemcpyAsync(h.data(), m->sqerr, h.size() * 8, hipMemcpyDeviceToHost, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  double se = 0.0, mx = -1e300;
  for (int b = 0; b < nb; ++b) {
    se += h[2 * b];
    mx = std::max(mx, h[2 * b + 1]);
  }
  const double mse = se / (double)n;
  *psnr_host = mse == 0.0 ? INFINITY : 10.0 * std::log10(mx * mx / mse);
  return NIC_OK;
}

nic_status nic_psnr_noalloc(const float* gt_dev, const float* pred_dev, int64_t n, void* hip_stream,
                            double* psnr_host) {
  if (!gt_dev || !pred_dev || !psnr_host) return fail(NIC_EINVAL, "NULL argument");
  if (n < 1) return fail(NIC_EINVAL, "n must be >= 1");
  if (n > (int64_t)kNoAllocBlocks * kNoAllocPerBlock)
    return fail(NIC_EINVAL, "n = %lld exceeds the static scratch of nic_psnr_noalloc (at most %lld voxels)",
                (long long)n, (long long)kNoAllocBlocks * kNoAllocPerBlock);
  double* part = nullptr;
  const nic_status st = scratch_address(&part);
  if (st != NIC_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const int nb = (int)((n + kNoAllocPerBlock - 1) / kNoAllocPerBlock);
  // every partial the host reads is written by this launch: nothing to clear
  NIC_HIP(launch_sqerr(gt_dev, pred_dev, n, part, nb, stream));
  thread_local double h[2 * kNoAllocBlocks];
  NIC_HIP(hipMemcpyAsync(h, part, (size_t)nb * 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
  NIC_HIP(hipStreamSynchronize(stream));
  double se = 0.0, mx = -1e300;
  for (int b = 0; b < nb; ++b) {
    se += h[2 * b];
    mx = std::max(mx, h[2 * b + 1]);
  }
  const double mse = se / (double)n;
  *psnr_host = mse == 0.0 ? INFINITY : 10.0 * std::log10(mx * mx / mse);
  return NIC_OK;
}

nic_status nic_ssim(nic_model* m, const float* gt_dev, const float* pred_dev, const int32_t dims[3],
                    double* ssim_host) {
  if (!model_ok(m) || !gt_dev || !pred_dev || !dims || !ssim_host) return fail(NIC_EINVAL, "NULL argument");
  for (int k = 0; k < 3; ++k)
    if (dims[k] < 11 || dims[k] > 4096) return fail(NIC_EINVAL, "dims must be in [11, 4096] (11-voxel window)");
  const int64_t n = (int64_t)dims[0] * dims[1] * dims[2];
  const int64_t nv = (int64_t)(dims[0] - 10) * (dims[1] - 10) * (dims[2] - 10);
  // data range L = max(gt), from the PSNR kernel's per-block maxima
  const int nbm = (int)std::min<int64_t>(kSqerrBlocks, (n + 255) / 256);
  NIC_HIP(launch_sqerr(gt_dev, gt_dev, n, m->sqerr, nbm, m->stream));
  std::vector<double> h(2 * (size_t)kSqerrBlocks);
  NIC_HIP(hipMemcpyAsync(h.data(), m->sqerr, 2 * (size_t)nbm * 8, hipMemcpyDeviceToHost, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  double L = -1e300;
  for (int b = 0; b < nbm; ++b) L = std::max(L, h[2 * b + 1]);
  const double c1 = (0.01 * L) * (0.01 * L), c2 = (0.03 * L) * (0.03 * L);
  const int nb = (int)std::min<int64_t>(2 * kSqerrBlocks, (nv + 255) / 256);
  NIC_HIP(launch_ssim(gt_dev, pred_dev, dims[0], dims[1], dims[2], c1, c2, m->sqerr, nb, m->stream));
  NIC_HIP(hipMemcpyAsync(h.data(), m->sqerr, (size_t)nb * 8, hipMemcpyDeviceToHost, m->stream));
  NIC_HIP(hipStreamSynchronize(m->stream));
  double total = 0.0;
  for (int b = 0; b < nb; ++b) total += h[b];
  *ssim_host = total / (double)nv;
  return NIC_OK;
}

}  // extern "C"
