/*
 * nic.h - C ABI of libnic: training step of a hash-encoded attenuation field for sparse-view
 * cone-beam CT on one AMD MI355X (gfx950), following Xu et al., "NeRF-based CBCT Reconstruction
 * needs Normalization and Initialization" (arXiv 2506.19742).
 *
 * Problem statement (Sec. 2.1 Pipeline, Sec. 2.2): cone-beam projections with known source and
 * detector positions go in; an attenuation field mu(x, y, z), queried at points or rendered on a
 * voxel grid, comes out.  The field is a multiresolution hash encoding (Instant-NGP, cited in
 * Sec. 1), a LayerNorm (the "Normalized Hash Encoder", Sec. 2.3) and a small MLP.  Training
 * minimises the L1 distance between measured line integrals and the ray sums of Eq. (1)
 * (Sec. 2.5, Eq. 3) with Adam at lr 1e-3, one view per step (Sec. 3.1).  Mapping Consistency
 * Initialization transfers the LayerNorm + MLP weights of a trained model to a new one
 * (Sec. 2.1, Sec. 2.4).
 *
 * Conventions shared by every entry point:
 *  - Memory: the caller owns every device buffer.  All model state lives in one caller-provided
 *    device workspace of nic_workspace_size() bytes; the library never allocates device memory.
 *    Pointers named *_dev are device pointers, everything else is host memory.
 *  - Streams: every call is asynchronous on the stream given to nic_create (a hipStream_t, NULL =
 *    default stream), except those documented as synchronous (loss_host != NULL, export/import,
 *    save/load), which synchronise that stream before returning.
 *  - Errors: a negative nic_status; nic_last_error() returns a message (thread-local).  Argument
 *    errors (NIC_EINVAL) are detected before any launch and leave the model unchanged.  No
 *    exception or abort crosses the ABI.
 *  - Threading: calls on one model must not overlap; use one model per host thread and stream.
 *
 * Geometry (all lengths mm, rotation about z): source s = dso (cos a, sin a, 0); detector centre
 * -(dsd - dso)(cos a, sin a, 0); detector axes e_u = (-sin a, cos a, 0), e_v = (0, 0, 1); pixel
 * (row r, column c) centre at u = ((c + 1/2) - nu/2) du + off_u, v = ((r + 1/2) - nv/2) dv + off_v.
 * Projections are line integrals A = -ln(I/I0) (Eq. 1), float32 [n_views][nv][nu], pixel index
 * r * nu + c.  The reconstruction box [-vol/2, vol/2] is centred at the origin; normalised
 * coordinates are x_n = (x + vol/2) / vol in [0, 1].
 */
#ifndef NIC_H
#define NIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nic_status;
#define NIC_OK 0
#define NIC_EINVAL (-1)      /* invalid argument or unsupported configuration */
#define NIC_ENOMEM (-2)      /* workspace too small */
#define NIC_EHIP (-3)        /* HIP runtime error (launch or copy) */
#define NIC_ENONFINITE (-4)  /* a non-finite value met (projections, loss, residual, gradient) */
#define NIC_EVERSION (-5)    /* blob or state of another format/version/configuration */
#define NIC_ESTATE (-6)      /* call not valid in the model's current state */

typedef struct nic_geometry {
  double dso, dsd;            /* source-origin, source-detector distance (mm), dsd > dso > 0 */
  int32_t det_nu, det_nv;     /* detector columns, rows (>= 1) */
  double det_du, det_dv;      /* pixel pitch (mm, > 0) */
  double det_off_u, det_off_v;/* detector offset (mm) */
  double vol_size[3];         /* box edge lengths x, y, z (mm, > 0) */
  int32_t n_views;            /* >= 1 */
  int32_t pad_;
  const double* angles_rad;   /* host [n_views], copied by nic_create */
} nic_geometry;

typedef struct nic_config {
  /* Encoder (multiresolution hash grid, Instant-NGP as cited in Sec. 1): L levels, F = 2 features
   * per level, T = 2^log2_table entries per hashed level (4 <= log2_table <= 26), resolutions
   * N_l = floor(N_min b^l) with b = exp((ln N_max - ln N_min)/(L-1)), 1 <= N_min <= N_max <= 32768.
   * Supported: L in {8, 16}, F == 2. */
  int32_t n_levels, feats_per_level, log2_table, base_res, max_res;
  /* Network: depth hidden ReLU layers of width W, linear head.  Supported (W, depth): W = 32 with
   * 1 <= depth <= 4, and W = 64 with depth 4.  out_act 0: mu = mu_max * sigmoid(y), 1: identity
   * (mu = y), 2: softplus (beta 1, threshold 20: mu = y above 20).  Anything else is NIC_EINVAL. */
  int32_t mlp_depth, mlp_width, out_act;
  /* Samples per ray N (multiple of 32, 32..1024) and rays per step R (1..65536, <= pixels). */
  int32_t samples_per_ray, rays_per_step;
  int32_t layernorm;          /* 1: LayerNorm between encoder and network (Sec. 2.3), 0: none */
  int32_t precision;          /* 0: FP32; 1: BF16 MLP operands (FP32 accumulate) + FP16 table
                                 copy for gathers, FP32 master weights, grads and Adam */
  int32_t n_tables;           /* K hash tables sharing one LayerNorm + MLP (pre-training for
                                 Mapping Consistency Initialization, Sec. 2.4); 0 or 1 = one table.
                                 Ray training and rendering use table 0. */
  int32_t pad_;
  double mu_max;              /* output scale for out_act 0 (1/mm) */
  double ln_eps;              /* LayerNorm epsilon */
  double lr, beta1, beta2, adam_eps;   /* Adam (Sec. 3.1: lr 1e-3) */
  uint64_t seed;              /* Philox4x32-10 key for the device draws */
} nic_config;

/* Host-side description of a configuration (no GPU needed). */
typedef struct nic_layout {
  int32_t n_levels;
  int32_t res[16];            /* N_l */
  int32_t dense[16];          /* 1 when the level stores one entry per vertex */
  int64_t offset[16];         /* first entry of the level */
  int64_t n_entries;          /* entries of one table (each feats_per_level floats) */
  int64_t n_table;            /* table parameters = n_tables * n_entries * feats_per_level */
  int64_t n_dense;            /* LayerNorm + MLP parameters */
  int64_t dense_offset;       /* index of the first dense parameter in the parameter vector */
  int64_t n_params_padded;    /* length of the parameter vector (padding entries stay 0) */
  int32_t bin_shift;          /* table-gradient bins span 2^bin_shift entries (>= 13) */
  int32_t n_bins;             /* bins over all tables */
} nic_layout;

typedef struct nic_model nic_model;   /* opaque; owns no device memory */

/* Tensor view returned by nic_tensors. dtype 0 = float32, 1 = float16. */
typedef struct nic_tensor {
  void* ptr;
  int64_t numel;
  int32_t dtype;
  int32_t pad_;
} nic_tensor;

/* Level table and parameter counts of a configuration.  Parameter vector layout:
 * [tables: n_tables x n_entries x F, entry-major, level after level][padding][dense block][padding], dense
 * block = ln_gain[C] ln_bias[C] then per hidden layer k: W_k[W][in_k] (row = output unit) b_k[W],
 * then w_out[W] b_out[1], with C = L*F, in_0 = C, in_k = W.  Returns NIC_EINVAL for an
 * unsupported configuration.  Host only. */
nic_status nic_describe(const nic_config* cfg, nic_layout* out);

/* Bytes of device workspace a model needs (0 for an invalid configuration).  Host only. */
size_t nic_workspace_size(const nic_config* cfg, const nic_geometry* geom);

/* Creates a model in the caller's workspace (>= nic_workspace_size bytes, 256-byte aligned) on
 * hip_stream, and initialises the parameters on the device from cfg->seed (table uniform in
 * [-1e-4, 1e-4), linear layers uniform in +-1/sqrt(fan_in), LayerNorm gain 1 bias 0; Adam state 0,
 * step 0).  The host object is freed by nic_destroy; the workspace stays the caller's. */
nic_status nic_create(const nic_config* cfg, const nic_geometry* geom, void* hip_stream,
                      void* workspace, size_t ws_bytes, nic_model** out);
void nic_destroy(nic_model* m);

/* Message of the last failing call on this thread ("" if none). */
const char* nic_last_error(void);

/* Borrows the measured projections (device, float32 [n_views][nv][nu] line integrals) until
 * nic_destroy or the next call.  Synchronous: every value is checked first; NIC_ENONFINITE (and the
 * previous projections stay in use) when any is NaN or infinite, NIC_EINVAL for NULL. */
nic_status nic_set_projections(nic_model* m, const float* proj_dev);

/* Non-finite values met during training.  A training call (nic_step, nic_train, nic_backward,
 * nic_adam, nic_voxel_step, nic_voxel_train) whose step meets a NaN or infinite loss, ray residual,
 * upstream gradient, table-gradient contribution or per-block network gradient writes no parameter,
 * Adam moment or gradient; from then on every later step is skipped the same way (the model stays
 * bitwise as it was before that step) until the host learns of it at the next synchronising check:
 * nic_sync, nic_train / nic_voxel_train with loss_host != NULL, or nic_save_state.  That check returns
 * NIC_ENONFINITE, sets the step counter back to the first skipped step, and clears the condition, so
 * training can go on from there (for example after the projections were fixed).
 * nic_sync: synchronises the model's stream and performs that check (NIC_OK when nothing was met). */
nic_status nic_sync(nic_model* m);

/* Device views of the parameters, gradients and Adam moments, in this order: params (float32,
 * n_params_padded), grads, adam_m, adam_v, table_f16 (float16, n_table; precision 1 only, else
 * numel 0).  *count receives 5.  Writing params directly is allowed between calls (call
 * nic_sync_params afterwards when precision == 1). */
nic_status nic_tensors(nic_model* m, nic_tensor* out, int32_t* count);

/* Re-derives the FP16 table copy from the FP32 master table (precision 1; no-op otherwise). */
nic_status nic_sync_params(nic_model* m);

/* Re-initialises parameters from seed (as in nic_create) and resets Adam state and step to 0. */
nic_status nic_init_params(nic_model* m, uint64_t seed);

/* One full training step (Sec. 2.5, Eq. 3; Sec. 3.1): rays of one view -> samples -> encode ->
 * LayerNorm -> MLP -> ray sums (Eq. 1) -> L1 loss -> backward (table scatter-add, MLP and
 * LayerNorm gradients) -> Adam on every parameter.  view in [0, n_views).  pix_dev: device int32
 * [R] distinct pixel indices, or NULL to draw them on the device (Philox, step counter as
 * counter).  jitter_dev: device float32 [R][N] in [0, 1), or NULL to draw on the device.
 * loss_dev: device float32 [1] receiving the step's loss, or NULL.  Increments the step. */
nic_status nic_step(nic_model* m, int32_t view, const int32_t* pix_dev, const float* jitter_dev,
                    float* loss_dev);

/* n_steps training steps with every draw on the device: view order a fresh permutation of the
 * views per epoch of n_views steps, pixels and jitter from Philox.  loss_host: host float32
 * [n_steps] (synchronous; NIC_ENONFINITE if any loss is not finite or a step was skipped, see
 * nic_sync) or NULL (asynchronous; a skipped step is reported by the next check).  One call of n
 * steps equals n calls of one step bit for bit; within a call each step's last kernel also draws
 * the next step's rays, so a call of many steps saves a launch per step. */
nic_status nic_train(nic_model* m, int32_t n_steps, float* loss_host);

/* The view nic_train uses at step `step` (host only). */
int32_t nic_view_for_step(const nic_model* m, int64_t step);

/* The pixels and jitter the device draws at step `step` (as nic_step with NULL arrays). */
nic_status nic_draw_rays(nic_model* m, int64_t step, int32_t* pix_dev, float* jitter_dev);

/* Forward pass only (Eq. 1): a_pred_dev (device float32 [n_rays]) = ray sums of n_rays rays of
 * `view` with the given pixels and jitter (both required). 0 <= n_rays <= rays_per_step, else
 * NIC_EINVAL; n_rays == 0 does nothing (the pointers are not used). */
nic_status nic_forward(nic_model* m, int32_t view, const int32_t* pix_dev, const float* jitter_dev,
                       int32_t n_rays, float* a_pred_dev);

/* Backward pass for an upstream gradient dA_dev (device float32 [n_rays], d loss / d A_pred) of
 * the same rays: accumulates parameter gradients into the grads tensor (not zeroed first).
 * Same n_rays rules as nic_forward. */
nic_status nic_backward(nic_model* m, int32_t view, const int32_t* pix_dev, const float* jitter_dev,
                        int32_t n_rays, const float* dA_dev);

/* Adam step on every parameter (dense, PyTorch semantics), then zeroes the gradients and
 * increments the step. */
nic_status nic_adam(nic_model* m);

/* Zeroes the gradients. */
nic_status nic_zero_grad(nic_model* m);

/* mu at n points given in normalised coordinates (device float32 [n][3] in [0, 1]) into mu_dev
 * (device float32 [n]).  n == 0 does nothing; n < 0 is NIC_EINVAL. */
nic_status nic_query(nic_model* m, const float* xn_dev, int64_t n, float* mu_dev);

/* Channel mask (Sec. 2.3: channels of the hash features that carry only noise, found with an FFT,
 * are masked during training): from this call on, every forward and backward pass feeds
 * mask_host[c] * (channel c of the encoding) to LayerNorm, c = level * 2 + feature; the table
 * entries of a channel with mask 0 receive no gradient.  mask_host: host float32 [n], n must be
 * n_levels * 2; copied.  NULL removes the mask.  Not part of saved states or MLP blobs. */
nic_status nic_set_channel_mask(nic_model* m, const float* mask_host, int32_t n);

/* Spectral noise measure of every hash-feature channel, the FFT criterion behind the channel mask
 * (Sec. 2.3): for level l of resolution N, the channel's field at the G^3 vertices v0 + i,
 * G = min(g_max, N), v0 = (N - G) / 2 (centre of the box), from the FP32 table of the first hash
 * table; 3-D DFT in FP64; hf_host[2l + f] (host float32 [n_levels * 2]) = power with
 * max_d |k_d| > G/4 over all non-DC power (about 0.875 for white noise, near 0 for a smooth field).
 * g_max in [4, 64]; uses the record buffer as scratch; synchronous. */
nic_status nic_channel_spectrum(nic_model* m, int32_t g_max, float* hf_host);

/* The feature-to-attenuation mapping alone (Sec. 2.3; Fig. 3 studies how it drifts for fixed
 * features during training): LayerNorm (when enabled), MLP and output activation applied to n given
 * encoder outputs enc_dev (device float32 [n][n_levels * 2], channel l * 2 + f, the layout
 * nic_encode writes), into mu_dev (device float32 [n]).  Asynchronous on the model's stream. */
nic_status nic_field_from_features(nic_model* m, const float* enc_dev, int64_t n, float* mu_dev);

/* mu at the voxel centres ((i + 1/2)/nx, (j + 1/2)/ny, (k + 1/2)/nz) into vol_dev (device float32
 * [nz][ny][nx]); dims = {nx, ny, nz}. */
nic_status nic_render_volume(nic_model* m, const int32_t dims[3], float* vol_dev);

/* Raw encoding (before LayerNorm) at n normalised points, gathered from the table the forward pass
 * uses (FP32, or the FP16 copy when precision == 1): enc_dev (device float32 [n][L*F], channel
 * l*F + f) and, when idx_dev != NULL, the global table entry of every corner (device uint32
 * [n][L][8], corner c = c0 + 2 c1 + 4 c2). */
nic_status nic_encode(nic_model* m, const float* xn_dev, int64_t n, float* enc_dev, uint32_t* idx_dev);

/* Voxel loss step for the pre-training of Mapping Consistency Initialization (Sec. 2.1 and
 * Sec. 2.4, Eq. 2): n_points points of the unit cube, split into n_tables equal contiguous groups
 * (point p uses table p / (n_points / n_tables)), target mu = trilinear sample of that table's volume
 * (set by nic_set_volumes), loss = mean |mu - target|, then backward and Adam as in nic_step.
 * xn_dev: device float32 [n_points][3] in [0, 1], or NULL to draw the points on the device
 * (Philox, step counter as counter).  n_points must be a multiple of 32 * n_tables and at most
 * rays_per_step * samples_per_ray.  loss_dev: device float32 [1] or NULL.  Increments the step. */
nic_status nic_voxel_step(nic_model* m, const float* xn_dev, int32_t n_points, float* loss_dev);

/* n_steps voxel steps with device-drawn points; loss_host as in nic_train. */
nic_status nic_voxel_train(nic_model* m, int32_t n_steps, int32_t n_points, float* loss_host);

/* Borrows the pre-training target volumes: device float32 [n_tables][n][n][n] (z, y, x order,
 * voxel-centre sampling, n >= 2). */
nic_status nic_set_volumes(nic_model* m, const float* vols_dev, int32_t n);

/* Mapping Consistency Initialization transfer (Sec. 2.1, Sec. 3.1): only the LayerNorm and MLP
 * weights move between models.  nic_export_mlp writes a host blob (header + FP32 dense block);
 * with buf == NULL it only stores the size in *bytes.  nic_import_mlp loads a blob of a model with
 * the same channel count, width, depth, output activation, LayerNorm flag, output scale mu_max and
 * LayerNorm epsilon into the dense block and resets its Adam moments (the hash table keeps its own
 * values).  Both synchronise the stream; NIC_EVERSION for a blob of another format or network. */
nic_status nic_export_mlp(nic_model* m, void* buf, size_t* bytes);
nic_status nic_import_mlp(nic_model* m, const void* buf, size_t bytes);

/* Checkpoint and resume: the full training state (parameters, Adam moments, step counter; the
 * device draws are counter-based, so the step and the seed define the rest) as a host blob with a
 * header naming the configuration.  nic_save_state with buf == NULL stores the size in *bytes;
 * it returns NIC_ENONFINITE without saving when a step was skipped (see nic_sync; call again to
 * save the state as it stands after that check).
 * nic_load_state requires the same configuration and seed (NIC_EVERSION otherwise), zeroes the
 * gradients and refreshes the FP16 table copy.  A resumed run reproduces an uninterrupted one bit
 * for bit.  Both synchronise the stream. */
nic_status nic_save_state(nic_model* m, void* buf, size_t* bytes);
nic_status nic_load_state(nic_model* m, const void* buf, size_t bytes);

/* PSNR = 10 log10(max(gt)^2 / mean((pred - gt)^2)) over n voxels (device float32 arrays); the
 * squared errors are summed in FP64 on the device; synchronous.  +inf when pred == gt. */
nic_status nic_psnr(nic_model* m, const float* gt_dev, const float* pred_dev, int64_t n, double* psnr_host);

/* nic_psnr without a model or workspace, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same PSNR of gt_dev
 * and pred_dev (device float32 [n], on the current device), on hip_stream (a stream of the current
 * device; NULL = its default stream); synchronous.  Allocates nothing: the per-block partial sums
 * go to a static device array of the library (4096 pairs of doubles, 64 KB, held on each device it
 * runs on until the process ends), one block per 65,536 voxels, so n <= 268,435,456 (a 645^3
 * volume); a larger n returns NIC_EINVAL before any launch.  Calls on one device share the array:
 * calls that overlap on one device race. */
nic_status nic_psnr_noalloc(const float* gt_dev, const float* pred_dev, int64_t n, void* hip_stream,
                            double* psnr_host);

/* 3-D SSIM (the structural similarity of Wang et al. 2004, which Sec. 3.1 uses with PSNR, taken
 * over volumes): local means, variances and covariance under a separable Gaussian window (sigma 1.5,
 * 11 taps per axis, weights summing to 1), C1 = (0.01 L)^2 and C2 = (0.03 L)^2 with L = max(gt), the
 * SSIM map averaged over the voxels whose whole window lies inside the volume.  gt_dev, pred_dev:
 * device float32 [dims[2]][dims[1]][dims[0]], every dim in [11, 4096].  FP64 on the device;
 * synchronous. */
nic_status nic_ssim(nic_model* m, const float* gt_dev, const float* pred_dev, const int32_t dims[3],
                    double* ssim_host);

/* Current Adam step count (host only). */
int64_t nic_get_step(const nic_model* m);

/* Encoder placement of the ray training steps (nic_train, nic_step, nic_backward) on a model with
 * one table.  NIC_ENCODER_LEVEL_MAJOR: a level-major encoder kernel computes the hash encoding
 * (Sec. 2.2) and the gradient-record counts, with each XCD of the chip working on one level of the
 * grid at a time so that the level's table stays in that XCD's L2, and the forward kernel reads
 * the stored encoding.  NIC_ENCODER_IN_FORWARD: the forward kernel gathers all levels itself.
 * NIC_ENCODER_AUTO (the default): level-major when the whole table (8 B per entry, 4 B in the
 * precision form) exceeds the device's L2 size and no level's table exceeds twice it.  All give
 * bitwise identical results (same arithmetic in the same order).  Every other pass (queries,
 * rendering, pre-training) always encodes inside its own kernel.  nic_encoder_level_major returns 1
 * when the training steps of m currently use the level-major encoder (0 for a NULL model).
 * Errors: NIC_EINVAL for a NULL model or another placement value. */
#define NIC_ENCODER_AUTO 0
#define NIC_ENCODER_LEVEL_MAJOR 1
#define NIC_ENCODER_IN_FORWARD 2
nic_status nic_set_encoder_placement(nic_model* m, int32_t placement);
int32_t nic_encoder_level_major(const nic_model* m);

/* Kernel timing for benchmarks: with enable != 0, every kernel of the training path is bracketed
 * by a pair of HIP events on the model's stream.  nic_kernel_times synchronises the stream and
 * returns, per kernel kind k (0 rays (in nic_train the first step of a call only), 1 forward,
 * 2 backward, 3 encode (the level-major encoder), 4 adam, 5 bin scan, 6 bin reduce, which includes
 * the dense reduction and, in nic_train, the next step's ray draw), the total milliseconds
 * ms[k] and the number of launches calls[k] since timing was enabled; ms and calls must hold at
 * least 7 entries (*count = 7, the number written). */
nic_status nic_set_timing(nic_model* m, int32_t enable);
nic_status nic_kernel_times(nic_model* m, double* ms, int64_t* calls, int32_t* count);

#ifdef __cplusplus
}
#endif

#endif /* NIC_H */
