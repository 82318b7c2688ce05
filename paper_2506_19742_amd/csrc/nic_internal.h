// Kernel argument blocks and launch entry points shared by the kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "nic_device.h"

namespace nic {

enum { kModeRays = 0, kModePoints = 1, kModeVoxels = 2, kModeVoxelLoss = 3, kModeFeatures = 4 };

struct FwdArgs {
  int32_t mode;          // kModeRays / kModePoints / kModeVoxels
  int32_t N;             // samples per ray (rays mode)
  int64_t n_points;      // rays: n_rays * N
  const void* table;     // table gathered by the forward: FP32 [n_entries][2], or FP16 (precision 1)
  const float* dense;    // FP32 dense parameters (global layout)
  LevelTab lt;
  Geo geo;
  const RayRec* rays;
  const float* jitter;   // [n_rays][N] or NULL (Philox)
  uint64_t seed;
  uint32_t step;
  int32_t layernorm;
  int32_t out_act;
  float mu_max;
  float ln_eps;
  const float* mask;     // [C] channel mask applied before LayerNorm, or NULL (raw encoding stored)
  int32_t dims[3];       // voxel grid (voxels mode)
  const float* xn;       // points mode [n][3]
  const float* feats;    // features mode: encoder outputs [n][2L], channel l * 2 + f
  float* enc_out;        // rays mode: raw encoding, lane-major per wave (or NULL)
  const float* enc_pre;  // rays mode: raw encoding already computed by k_enc, same layout (or NULL)
  float* wave_sum;       // rays mode: per-wave partial sums of mu * delta
  float* mu_out;         // points / voxels mode
  uint32_t* bin_counts;  // training: [n_bins][gridDim] records per (bin, block), or NULL
  int32_t n_bins;
  // k_enc: backward grid G, and the counts of each level's first and last bin, [2L][G] (a bin at a
  // level boundary can hold entries of several levels; the bin scan adds these rows)
  int32_t enc_grid;
  uint32_t* edge_counts;
  // k_fwd reading k_enc's encoding: the record offsets' row scans of k_enc's counts (bin_row_scan
  // over bins blockIdx, blockIdx + gridDim, ...; no separate k_bin_rowscan), or scan_rel == NULL
  const uint32_t* scan_counts;
  uint32_t* scan_rel;
  uint32_t* scan_totals;
  const int32_t* edge_beg;
  const int32_t* edge_src;
  // voxel-loss mode (pre-training): point p uses table p / pts_per_table, whose entries start at
  // (p / pts_per_table) * table_stride, and the target volume of that table
  int64_t pts_per_table;
  uint32_t table_stride;
  int32_t vol_n;
  const float* vols;     // [n_tables][vol_n]^3
};

struct BwdArgs {
  const float* enc_in;   // encoding stored by k_fwd
  const float* dA_in;    // [n_rays] upstream gradient, or NULL for the L1 loss of Eq. (3)
  float inv_R;           // 1/R for the mean over rays
  float* a_pred_out;     // [n_rays] (L1 mode)
  float* absres_out;     // [n_rays] (L1 mode)
  float* partials;       // [grid][nd_pad] per-block dense gradients
  const uint32_t* bin_offsets;  // [n_bins][grid] first slot of each (bin, block) run within the bin
  const uint32_t* bin_start;    // [n_bins] first record of each bin
  BinRec* recs;          // table-gradient records grouped by bin
  uint32_t rec_cap;      // capacity of recs: a slot at or beyond it is not written (and flagged)
  float* wave_loss;      // voxel-loss mode: per-wave sum of |mu - target|
  uint32_t* rec_max_bits;  // bit pattern of the largest |record| of the step (atomic max)
  uint32_t* bad_step;    // 0, or 1 + the first step that met a non-finite value (sticky)
};

struct RaysArgs {
  Geo geo;
  double ca, sa;         // cos, sin of the view angle (host libm)
  int32_t view;
  int32_t N;
  int32_t n_rays;
  int32_t h_bits;        // Feistel half width
  uint32_t n_pix;
  uint32_t step;
  uint64_t seed;
  const int32_t* pix_in; // or NULL: device draw
  const float* proj;     // [n_views][n_pix] or NULL
  RayRec* rays;
  int32_t* pix_out;      // optional
  float* jitter_out;     // optional [n_rays][N]
};

struct InitArgs {
  uint64_t seed;
  int64_t n_dense;
  int64_t ln_end;          // 2C
  int64_t first_layer_end; // end of W_0, b_0
  int32_t fan0;            // C
  int32_t width;           // W
};

struct KernelSet {
  const void* fwd = nullptr;
  const void* bwd = nullptr;
  const void* enc = nullptr;
  const void* fwd_pre = nullptr;   // k_fwd reading the encoding stored by k_enc
  size_t fwd_lds = 0, bwd_lds = 0;
  int n_dense = 0, nd_pad = 0;
  bool valid = false;
};

KernelSet kernel_set(int L, int W, int D, int precision);
// Forward: grid = min(chunks, max_grid) persistent blocks (max_grid <= 0: one block per chunk);
// extra_lds = bytes of the bin histogram when counting.
hipError_t launch_fwd(const KernelSet& ks, const FwdArgs& a, int max_grid, size_t extra_lds, hipStream_t s);
hipError_t launch_bwd(const KernelSet& ks, const FwdArgs& a, const BwdArgs& b, int grid, size_t extra_lds,
                      hipStream_t s);
// Level-major encoder of the rays mode (a.enc_out, a.bin_counts, a.edge_counts, a.enc_grid set):
// 8 * ceil(L / 8) * a.enc_grid blocks; lds = bytes of the largest level's bin histogram.
hipError_t launch_enc(const KernelSet& ks, const FwdArgs& a, size_t lds, hipStream_t s);
hipError_t launch_rays(const RaysArgs& a, hipStream_t s);
hipError_t launch_raysum(const float* wave_sum, int waves_per_ray, int n_rays, float* out, hipStream_t s);
// Adam over all n parameters from the stored gradient (gradient reset to 0).
// Skipped (nothing written) when *bad_step != 0.
hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float ibc1, float ibc2, __half* th, int64_t n_table, const uint32_t* bad_step,
                       int n_cu, hipStream_t s);
// Number of non-finite values among x[0 .. n) into *count (u32, overwritten).
hipError_t launch_count_nonfinite(const float* x, int64_t n, uint32_t* count, int n_cu, hipStream_t s);
hipError_t launch_fill(float* x, int64_t n, float val, int n_cu, hipStream_t s);
hipError_t launch_to_half(const float* src, __half* dst, int64_t n, int n_cu, hipStream_t s);
hipError_t launch_init(float* params, int64_t n_table, int64_t dense_off, const InitArgs& ia, int n_cu,
                       hipStream_t s);
// bin_start: [n_bins + 1]; block_start: [reduce_grid + 1] record ranges of the bin reduction's blocks.
// edge (k_enc's counts): when not NULL, bin b with edge_beg[b] < edge_beg[b + 1] takes its per-block
// counts as the sum of the rows edge[edge_src[k] * grid ..] for k in that range, not from counts.
hipError_t launch_bin_scan(const uint32_t* counts, int n_bins, int grid, uint32_t* rel, uint32_t* totals,
                           uint32_t* bin_start, uint32_t* block_start, int32_t* block_first_bin, int reduce_grid,
                           uint32_t* rec_max_bits, const uint32_t* edge, const int32_t* edge_beg,
                           const int32_t* edge_src, bool rows_done, hipStream_t s);
// Dense (LayerNorm + MLP) gradient reduction run by the last blocks of k_bin_combine.
struct DenseReduceArgs {
  const float* partials;   // [n_blocks][nd_pad] per-block partial sums from k_bwd
  int32_t n_blocks, nd_pad, nd;
  float* grad_dense;       // [nd]
  const float* absres;     // [n_rays] |residual| per ray (or per wave), or NULL
  int32_t n_rays;
  float inv_R;
  float* loss_out;         // loss = sum absres * inv_R, or NULL
  int32_t fused;           // Adam on p/m/v (gradient left at zero) instead of grad_dense += sum
  AdamArgs adam;
  float* p;                // dense parameters and Adam moments [nd]
  float* m;
  float* v;
  const uint32_t* bad_step;  // non-zero: a non-finite value was met, no parameter or gradient is written
};
struct BinReduceArgs {
  const BinRec* recs;             // records grouped by bin
  const uint32_t* bin_start;      // [n_bins + 1] first record of each bin; [n_bins] = total
  const uint32_t* block_start;     // [G' + 1] first record of each block's range, G' = min(grid, records)
  const int32_t* block_first_bin; // [grid] bin holding the first record of each block's range
  int32_t n_bins;
  int32_t bin_shift;              // log2 entries per bin
  int32_t n_sub;                  // 2^(bin_shift - kBinBits) LDS tiles per bin
  int32_t pad_;
  const uint32_t* rec_max_bits;   // largest |record| of the step (float bits)
  float* grad_table;              // FP32 table gradient, [n_entries][2]
  int64_t n_entries;
  unsigned long long* split_acc;  // [2 grid][n_sub][2 << kBinBits] int64 tiles of bins cut by range boundaries
  // Fused Adam (training steps whose gradients start at zero): the table gradient is never stored;
  // each entry's gradient goes straight into Adam on p/m/v (and the FP16 copy th when not NULL).
  int32_t fused;
  AdamArgs adam;
  float* p;                       // table parameters, Adam moments [n_entries][2]
  float* m;
  float* v;
  __half* th;
  const uint32_t* bad_step;       // non-zero: a non-finite value was met, nothing is written
  DenseReduceArgs dense;
  int32_t dense_blocks;           // (dense.nd + 63) / 64 extra k_bin_combine blocks
  // The next training step's ray batch, drawn by ray_blocks = ceil(n_rays / 1024) k_bin_combine
  // blocks placed first (none when next_rays.n_rays == 0): the ray buffer is free once k_bwd is done.
  RaysArgs next_rays;
  int32_t ray_blocks;
};
hipError_t launch_bin_reduce(const BinReduceArgs& a, int grid, hipStream_t s);
size_t bin_reduce_lds();
const void* bin_reduce_kernel(bool fused);   // the fused-Adam or the gradient-only form
hipError_t launch_probe_points(int N, int v0, int G, float* xn, hipStream_t s);
hipError_t launch_channel_power(const float* enc, int C, int c, int G, double2* b0, double2* b1, double* partials,
                                int n_blocks, hipStream_t s);
hipError_t launch_ssim(const float* gt, const float* pred, int nx, int ny, int nz, double c1, double c2,
                       double* partials, int n_blocks, hipStream_t s);
hipError_t launch_sqerr(const float* gt, const float* pred, int64_t n, double* partials, int n_blocks,
                        hipStream_t s);
hipError_t launch_encode(const LevelTab& lt, const void* table, int half_table, const float* xn, int64_t n,
                         float* enc, uint32_t* idx, hipStream_t s);

}  // namespace nic
