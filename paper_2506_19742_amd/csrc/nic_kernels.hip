// Kernels of the training step for gfx950 (one MI355X).
//
// Step = k_rays -> [k_enc ->] k_fwd -> bin scan -> k_bwd -> k_bin_reduce -> k_bin_combine on the
// model's stream.
//  k_rays   one thread per ray slot: pixel (given or Philox/Feistel draw), FP64 ray setup, A_gt.
//           Within a multi-step training call the first blocks of each step's k_bin_combine draw
//           the next step's rays instead.
//  k_enc    (ray training on one table whose levels fit an XCD's L2) level-major hash encoding,
//           one level per XCD at a time, and the per-bin record counts; k_fwd then reads it.
//  k_fwd    four waves per block, 32 points per wave, two lanes per point (lane half h handles
//           half of the levels): sample position -> hash encode (8 corner gathers per level) ->
//           LayerNorm -> MLP on v_mfma_f32_32x32x2f32 -> mu -> per-wave partial ray sum of
//           mu * delta (Eq. 1).  Stores the raw encoding lane-major for the backward pass.
//  k_bwd    persistent blocks over 128-point chunks: reloads the encoding, recomputes LayerNorm and
//           the MLP forward, reads the ray's sum -> dA = sign(A - A_gt)/R (Eq. 3) -> MLP backward
//           on MFMA (data gradients chained in registers, weight gradients via per-wave LDS
//           transposes), LayerNorm backward, then writes the corner gradients as records
//           (entry, w * g) at the block's slots of their gradient bins.  Dense (LayerNorm + MLP)
//           gradients accumulate in LDS and are written once per block as partial sums.
//  k_bin_reduce / k_bin_combine sum the table-gradient records bin by bin (exact fixed point) and,
//           in a training step, run Adam on the table; the last blocks of k_bin_combine sum the
//           per-block dense partials and run Adam on LayerNorm + MLP, and form the loss.
//  k_adam   (after a backward pass that left its gradients stored) one streaming pass over every
//           parameter: Adam update, gradient reset to 0.
#include <cfloat>

#include "nic_device.h"
#include "nic_internal.h"

namespace nic {

// ---------------------------------------------------------------------------------------------
// Dense parameter layout (global, in floats from the start of the dense block) and its LDS copy.
// Global: ln_g[C] ln_b[C] {W_k[W][K_k] b_k[W]}_k w_out[W] b_out.  LDS: weights padded to
// [W][K_k + 1] so both the forward (row-varying) and backward (column-varying) MFMA operand reads
// are free of bank conflicts.
// ---------------------------------------------------------------------------------------------
template <int C, int W, int D, int P>
struct Lay {
  static constexpr int K(int k) { return k == 0 ? C : W; }
  // global
  static constexpr int g_lng = 0, g_lnb = C;
  static constexpr int gW(int k) {
    int o = 2 * C;
    for (int i = 0; i < k; ++i) o += W * K(i) + W;
    return o;
  }
  static constexpr int gb(int k) { return gW(k) + W * K(k); }
  static constexpr int g_wo = gW(D), g_bo = gW(D) + W, g_n = gW(D) + W + 1;
  // LDS, FP32 form: weights padded to [W][K+1] followed by the bias of each layer
  static constexpr int sW(int k) {
    int o = 0;
    for (int i = 0; i < k; ++i) o += W * (K(i) + 1) + W;
    return o;
  }
  // LDS, BF16 form: MFMA operand blocks of 8 bf16 per lane (units of 4 floats), forward layout
  // then transposed (backward) layout, followed by the FP32 biases
  static constexpr int wf(int k) {
    int o = 0;
    for (int i = 0; i < k; ++i) o += (W / 32) * (K(i) / 16) * 64;
    return o;
  }
  static constexpr int wb(int k) {
    int o = wf(D);
    for (int i = 0; i < k; ++i) o += ((K(i) + 31) / 32) * (W / 16) * 64;
    return o;
  }
  static constexpr int n_w16 = wb(D);
  static constexpr int sb(int k) { return P ? 4 * n_w16 + k * W : sW(k) + W * (K(k) + 1); }
  static constexpr int s_small = P ? 4 * n_w16 + D * W : sW(D);
  static constexpr int s_lng = s_small, s_lnb = s_small + C, s_wo = s_small + 2 * C, s_bo = s_small + 2 * C + W;
  static constexpr int s_n = (s_small + 2 * C + W + 1 + 3) & ~3;
};

template <int C, int W, int D, int P>
__device__ void stage_params(const float* __restrict__ dense, float* __restrict__ sp) {
  using Ly = Lay<C, W, D, P>;
  const int t = threadIdx.x, nt = blockDim.x;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int Kk = Ly::K(k);
    if constexpr (P == 0) {
      for (int e = t; e < W * (Kk + 1); e += nt) {
        const int o = e / (Kk + 1), i = e - o * (Kk + 1);
        sp[Ly::sW(k) + e] = (i < Kk) ? dense[Ly::gW(k) + o * Kk + i] : 0.0f;
      }
    } else {
      __bf16* s16 = reinterpret_cast<__bf16*>(sp);
      // forward blocks: unit (mb, s, lane) holds W[32mb + lane%32][chan(8s + i, lane/32)], i < 8
      const int nf = (W / 32) * (Kk / 16) * 64 * 8;
      for (int e = t; e < nf; e += nt) {
        const int i = e & 7, q = e >> 3, lane = q & 63, ms = q >> 6;
        const int s = ms % (Kk / 16), mb = ms / (Kk / 16);
        const int o = 32 * mb + (lane & 31), col = chan(8 * s + i, lane >> 5);
        s16[8 * Ly::wf(k) + e] = (__bf16)dense[Ly::gW(k) + o * Kk + col];
      }
      // backward blocks: unit (ib, s, lane) holds W[chan(8s + i, lane/32)][32ib + lane%32]
      const int nb = ((Kk + 31) / 32) * (W / 16) * 64 * 8;
      for (int e = t; e < nb; e += nt) {
        const int i = e & 7, q = e >> 3, lane = q & 63, is = q >> 6;
        const int s = is % (W / 16), ib = is / (W / 16);
        const int o = chan(8 * s + i, lane >> 5), col = 32 * ib + (lane & 31);
        s16[8 * Ly::wb(k) + e] = (col < Kk) ? (__bf16)dense[Ly::gW(k) + o * Kk + col] : (__bf16)0.0f;
      }
    }
    for (int e = t; e < W; e += nt) sp[Ly::sb(k) + e] = dense[Ly::gb(k) + e];
  }
  for (int e = t; e < C; e += nt) {
    sp[Ly::s_lng + e] = dense[Ly::g_lng + e];
    sp[Ly::s_lnb + e] = dense[Ly::g_lnb + e];
  }
  for (int e = t; e < W; e += nt) sp[Ly::s_wo + e] = dense[Ly::g_wo + e];
  if (t == 0) sp[Ly::s_bo] = dense[Ly::g_bo];
}

// ---------------------------------------------------------------------------------------------
// Per-point pieces
// ---------------------------------------------------------------------------------------------

// Encoding of the levels handled by lane half h: register r = 4j + 2q + f holds feature f of level
// 4j + 2h + q, i.e. channel chan(r, h).
template <int L, int P>
__device__ __forceinline__ void encode_half(const LevelTab& T, const void* __restrict__ table_,
                                            const float x[3], int h, float e[L], bool count, uint32_t* hist,
                                            int ln, uint32_t tbase) {
#pragma unroll
  for (int j = 0; j < L / 4; ++j) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int lA = 4 * j + q, lB = 4 * j + 2 + q;
      if (!(((T.on >> lA) | (T.on >> lB)) & 1u)) {   // both levels of the pair unused: skip (wave-uniform)
        e[4 * j + 2 * q] = 0.0f;
        e[4 * j + 2 * q + 1] = 0.0f;
        continue;
      }
      const int32_t N = h ? T.res[lB] : T.res[lA];
      const uint32_t off = h ? T.off[lB] : T.off[lA];
      const uint32_t st = h ? T.stride[lB] : T.stride[lA];
      uint32_t idx[8];
      float w[8];
      uint32_t g0, g1, g2;
      level_corners(N, off + tbase, st, T.mask, x, idx, w, g0, g1, g2);
      float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        float2 v;
        if constexpr (P == 0) v = reinterpret_cast<const float2*>(table_)[idx[c]];
        else v = __half22float2(reinterpret_cast<const __half2*>(table_)[idx[c]]);
        s0 += w[c] * v.x;
        s1 += w[c] * v.y;
      }
      e[4 * j + 2 * q] = s0;
      e[4 * j + 2 * q + 1] = s1;
      if (count) {   // wave-uniform: the backward pass writes one record per corner per run
        bool cont, tail;
        run_flags(g0, g1, g2, ln, cont, tail);
        if (tail && hist) {
#pragma unroll
          for (int c = 0; c < 8; ++c) atomicAdd(hist + (idx[c] >> T.bin_shift), 1u);
        }
      }
    }
  }
}

// Corner contributions of the channel gradients gx (same layout as encode_half) as records
// (entry, w * g_f0, w * g_f1), each written at the next slot of this block's run for the entry's bin.
// Consecutive samples of the ray in the same cell (runs) share their 8 corner entries: a segmented
// scan over the half sums each run and only the run's last lane writes the 8 records.  A slot at or
// beyond rec_cap (only if the counts of the forward pass disagreed with the records) is not written;
// it sets vbits to the top pattern, which stops the step as a non-finite one.
template <int L>
__device__ __forceinline__ void scatter_half(const LevelTab& T, BinRec* __restrict__ recs, uint32_t* cursor,
                                             const float x[3], int h, const float gx[L], bool active, int ln,
                                             uint32_t tbase, uint32_t rec_cap, uint32_t& vbits) {
#pragma unroll
  for (int j = 0; j < L / 4; ++j) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int lA = 4 * j + q, lB = 4 * j + 2 + q;
      if (!(((T.on >> lA) | (T.on >> lB)) & 1u)) continue;   // both levels of the pair unused: no records
      // The half's level parameters are selected here, at each level pair: hoisted out of the chunk
      // loop they are spilled, and every reload of a spill waits for all the record stores before it.
      const int hq = opaque(h);
      const int32_t N = hq ? T.res[lB] : T.res[lA];
      const uint32_t off = hq ? T.off[lB] : T.off[lA];
      const uint32_t st = hq ? T.stride[lB] : T.stride[lA];
      uint32_t idx[8];
      float w[8];
      uint32_t g0, g1, g2;
      level_corners(N, off + tbase, st, T.mask, x, idx, w, g0, g1, g2);
      const float g0v = gx[4 * j + 2 * q], g1v = gx[4 * j + 2 * q + 1];
      float v0[8], v1[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        v0[c] = w[c] * g0v;
        v1[c] = w[c] * g1v;
      }
      bool cont, tail;
      run_flags(g0, g1, g2, ln, cont, tail);
      if (__ballot(cont) != 0) {            // wave-uniform: some lane continues a run
        // Segmented inclusive scan over each half-wave on DPP moves: Hillis-Steele steps 1, 2, 4, 8
        // inside each 16-lane row, then lanes 16..31 of the half add lane 15's sum when their run
        // reaches back into the first row.  start = first lane of this lane's run (the highest run
        // head at or below it, from the ballot of heads; lane 0 of a half always is one).  A step
        // that no lane of the wave takes (every run prefix shorter than its shift) is skipped: this
        // leaves every sum unchanged.
        const uint32_t heads = (uint32_t)(__ballot(!cont) >> (32 * h));
        const int start = 31 - __clz(heads & (0xFFFFFFFFu >> (31 - ln)));
        const int d = ln - start;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const float a0 = dpp_f<kDppRowShr + 1, 0xF>(v0[c]), a1 = dpp_f<kDppRowShr + 1, 0xF>(v1[c]);
          if (d >= 1) { v0[c] += a0; v1[c] += a1; }
        }
        if (__ballot(d >= 2) != 0) {
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const float a0 = dpp_f<kDppRowShr + 2, 0xF>(v0[c]), a1 = dpp_f<kDppRowShr + 2, 0xF>(v1[c]);
            if (d >= 2) { v0[c] += a0; v1[c] += a1; }
          }
        }
        if (__ballot(d >= 4) != 0) {
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const float a0 = dpp_f<kDppRowShr + 4, 0xF>(v0[c]), a1 = dpp_f<kDppRowShr + 4, 0xF>(v1[c]);
            if (d >= 4) { v0[c] += a0; v1[c] += a1; }
          }
        }
        if (__ballot(d >= 8) != 0) {
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const float a0 = dpp_f<kDppRowShr + 8, 0xF>(v0[c]), a1 = dpp_f<kDppRowShr + 8, 0xF>(v1[c]);
            if (d >= 8) { v0[c] += a0; v1[c] += a1; }
          }
        }
        if (__ballot(ln >= 16 && start <= 15) != 0) {
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const float a0 = dpp_f<kDppRowBcast15, 0xA>(v0[c]), a1 = dpp_f<kDppRowBcast15, 0xA>(v1[c]);
            if (ln >= 16 && start <= 15) { v0[c] += a0; v1[c] += a1; }
          }
        }
      }
      if (active && tail) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          vbits = max(vbits, max(__float_as_uint(fabsf(v0[c])), __float_as_uint(fabsf(v1[c]))));
          const uint32_t slot = atomicAdd(cursor + (idx[c] >> T.bin_shift), 1u);
          BinRec r;
          r.idx = idx[c];
          r.v0 = v0[c];
          r.v1 = v1[c];
          if (slot < rec_cap) recs[slot] = r;
          else vbits = 0xFFFFFFFFu;
        }
      }
    }
  }
}

// LayerNorm over the C channels of a point split across the two lane halves.
template <int C>
__device__ __forceinline__ void ln_forward(const float e[C / 2], const float* sp_g, const float* sp_b,
                                           float eps, int layernorm, int h, float xh[C / 2],
                                           float z[C / 2], float& rstd) {
  constexpr int RC = C / 2;
  if (!layernorm) {
#pragma unroll
    for (int r = 0; r < RC; ++r) { xh[r] = e[r]; z[r] = e[r]; }
    rstd = 1.0f;
    return;
  }
  float s = 0.0f;
#pragma unroll
  for (int r = 0; r < RC; ++r) s += e[r];
  s += xor32(s);
  const float mean = s * (1.0f / C);
  float v = 0.0f;
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    const float d = e[r] - mean;
    v += d * d;
  }
  v += xor32(v);
  rstd = 1.0f / sqrtf(v * (1.0f / C) + eps);
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    const int c = chan(r, h);
    xh[r] = (e[r] - mean) * rstd;
    z[r] = sp_g[c] * xh[r] + sp_b[c];
  }
}

// One hidden layer forward: out = relu(W x + b) for K inputs held as K/2 registers.
template <int K, int W>
__device__ __forceinline__ void layer_fwd(const float* __restrict__ sW, const float* __restrict__ sb,
                                          const float* xin, float* out, int lane) {
  const int m = lane & 31, h = lane >> 5;
  f32x16 acc[W / 32];
#pragma unroll
  for (int mb = 0; mb < W / 32; ++mb) acc[mb] = f32x16{};
#pragma unroll
  for (int s = 0; s < K / 2; ++s) {
    const float b = xin[s];
    const int col = chan(s, h);
#pragma unroll
    for (int mb = 0; mb < W / 32; ++mb) acc[mb] = mfma32(sW[(32 * mb + m) * (K + 1) + col], b, acc[mb]);
  }
#pragma unroll
  for (int R = 0; R < W / 2; ++R) {
    const float a = acc[R >> 4][R & 15] + sb[chan(R, h)];
    out[R] = a > 0.0f ? a : 0.0f;
  }
}

// Data gradient through one layer: gin = W^T g for KIN inputs (KIN/2 registers).
template <int KIN, int W>
__device__ __forceinline__ void layer_bwd_data(const float* __restrict__ sW, const float* g, float* gin,
                                               int lane) {
  const int m = lane & 31, h = lane >> 5;
  constexpr int IB = (KIN + 31) / 32;
  f32x16 acc[IB];
#pragma unroll
  for (int ib = 0; ib < IB; ++ib) acc[ib] = f32x16{};
#pragma unroll
  for (int s = 0; s < W / 2; ++s) {
    const float b = g[s];
    const int row = chan(s, h);
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) {
      const int i = 32 * ib + m;
      const float a = (i < KIN) ? sW[row * (KIN + 1) + i] : 0.0f;
      acc[ib] = mfma32(a, b, acc[ib]);
    }
  }
#pragma unroll
  for (int R = 0; R < KIN / 2; ++R) gin[R] = acc[R >> 4][R & 15];
}

// BF16 form of layer_fwd: v_mfma_f32_32x32x16_bf16, B operand = 8 consecutive registers of the lane
// (channels chan(8s + i, h)) rounded to bf16, A operand = one pre-arranged bf16x8 block per lane.
template <int K, int W>
__device__ __forceinline__ void layer_fwd_bf16(const bf16x8* __restrict__ wf, const float* __restrict__ sb,
                                               const float* xin, float* out, int lane) {
  const int h = lane >> 5;
  f32x16 acc[W / 32];
#pragma unroll
  for (int mb = 0; mb < W / 32; ++mb) acc[mb] = f32x16{};
#pragma unroll
  for (int s = 0; s < K / 16; ++s) {
    bf16x8 b;
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = (__bf16)xin[8 * s + i];
#pragma unroll
    for (int mb = 0; mb < W / 32; ++mb) acc[mb] = mfma32_bf16(wf[(mb * (K / 16) + s) * 64 + lane], b, acc[mb]);
  }
#pragma unroll
  for (int R = 0; R < W / 2; ++R) {
    const float a = acc[R >> 4][R & 15] + sb[chan(R, h)];
    out[R] = a > 0.0f ? a : 0.0f;
  }
}

template <int KIN, int W>
__device__ __forceinline__ void layer_bwd_data_bf16(const bf16x8* __restrict__ wb, const float* g, float* gin,
                                                    int lane) {
  constexpr int IB = (KIN + 31) / 32;
  f32x16 acc[IB];
#pragma unroll
  for (int ib = 0; ib < IB; ++ib) acc[ib] = f32x16{};
#pragma unroll
  for (int s = 0; s < W / 16; ++s) {
    bf16x8 b;
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = (__bf16)g[8 * s + i];
#pragma unroll
    for (int ib = 0; ib < IB; ++ib) acc[ib] = mfma32_bf16(wb[(ib * (W / 16) + s) * 64 + lane], b, acc[ib]);
  }
#pragma unroll
  for (int R = 0; R < KIN / 2; ++R) gin[R] = acc[R >> 4][R & 15];
}

// bf16 tile [32 rows][kTile16] (row = channel, column = point) for the weight-gradient MFMA.
constexpr int kTile16 = 40;

template <int NREG>
__device__ __forceinline__ void tile_put_bf16(__bf16* tile, const float* v, int blk, int lane) {
  const int n = lane & 31, h = lane >> 5;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int R = 16 * blk + r;
    if (R < NREG) tile[chan(r, h) * kTile16 + n] = (__bf16)v[R];
  }
}

// BF16 form of tile_outer: K = 32 points in two steps of 16, added to d.
__device__ __forceinline__ f32x16 tile_outer_bf16(const __bf16* tG, const __bf16* tH, int lane,
                                                  f32x16 d = f32x16{}) {
  const int m = lane & 31, h = lane >> 5;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(tG + m * kTile16 + 16 * s + 8 * h);
    const bf16x8 bb = *reinterpret_cast<const bf16x8*>(tH + m * kTile16 + 16 * s + 8 * h);
    d = mfma32_bf16(a, bb, d);
  }
  return d;
}

// Writes rows [32*blk, 32*blk + 32) of a per-point vector (n registers, layout chan) into a
// [32][kTile] tile with column = point.
template <int NREG>
__device__ __forceinline__ void tile_put(float* tile, const float* v, int blk, int lane) {
  const int n = lane & 31, h = lane >> 5;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int R = 16 * blk + r;
    if (R < NREG) tile[(chan(r, h)) * kTile + n] = v[R];
  }
}

// Sum over the 32 points of tile row m = lane % 32 (valid in every lane).
__device__ __forceinline__ float tile_rowsum(const float* tile, int lane) {
  const int m = lane & 31, h = lane >> 5;
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 16; ++j) s += tile[m * kTile + 16 * h + j];
  return s + xor32(s);
}

// G^T H over the 32 points of a tile pair, tG = G rows [32mb, 32mb+32), tH = H rows [32nb, ..),
// added to d: register r of lane (m, h) = entry (32mb + chan(r, h), 32nb + m).
__device__ __forceinline__ f32x16 tile_outer(const float* tG, const float* tH, int lane, f32x16 d = f32x16{}) {
  const int m = lane & 31, h = lane >> 5;
#pragma unroll
  for (int s = 0; s < 16; ++s) d = mfma32(tG[m * kTile + 16 * h + s], tH[m * kTile + 16 * h + s], d);
  return d;
}

// Cross-wave combination of the dense-gradient contributions of one chunk without float atomics
// (LDS float atomics are slow on gfx950): every wave stages its values in its own LDS slot, then
// each wave adds a disjoint quarter of the entries, summed over the four slots, to the block's
// accumulator.  Must be reached by all waves of the block.
struct Combine {
  float* slot0;        // slot of wave 0; wave w's slot is slot0 + w * stride
  int stride;
  int wv, lane;
  __device__ float* mine() const { return slot0 + wv * stride; }
  __device__ float sum4(int q) const {
    return slot0[q] + slot0[stride + q] + slot0[2 * stride + q] + slot0[3 * stride + q];
  }
  // dW block (mb, nb) of a layer with K inputs at acc[wbase]; optional 32 row sums (bias) staged
  // after the tile are added at acc[bbase + 32 mb + m] when bbase >= 0.
  __device__ void tile(float* acc, const f32x16& d, int wbase, int K, int mb, int nb, float brow, int bbase) const {
    float* S = mine();
#pragma unroll
    for (int r = 0; r < 16; ++r) S[r * kWave + lane] = d[r];
    if (lane < 32) S[1024 + lane] = brow;
    __syncthreads();
    const int ln = opaque(lane);   // addresses recomputed here rather than hoisted and spilled
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = 256 * wv + 64 * k + ln;
      const int r = q >> 6, l2 = q & 63, m2 = l2 & 31, h2 = l2 >> 5;
      const int col = 32 * nb + m2;
      if (col < K) acc[wbase + (32 * mb + chan(r, h2)) * K + col] += sum4(q);
    }
    if (bbase >= 0 && wv == 1 && lane < 32) acc[bbase + 32 * mb + lane] += sum4(1024 + lane);
    __syncthreads();
  }
  // The output unit's row sums (wo0 at wobase + m, wo1 at wobase + 32 + m when two32), the LayerNorm
  // gain and bias row sums (lg at gbase + m, lb at bbase + m for m < nrows; none when gbase < 0) and
  // the output bias (sc at scbase), combined in one staging round: each wave adds one of them.
  __device__ void rows_merged(float* acc, float wo0, float wo1, bool two32, int wobase, float lg, float lb,
                              int gbase, int bbase, int nrows, float sc, int scbase) const {
    float* S = mine();
    if (lane < 32) {
      S[lane] = wo0;
      S[32 + lane] = wo1;
      S[64 + lane] = lg;
      S[96 + lane] = lb;
    }
    if (lane == 0) S[128] = sc;
    __syncthreads();
    if (lane < 32) {
      if (wv == 0) acc[wobase + lane] += sum4(lane);
      if (wv == 1 && two32) acc[wobase + 32 + lane] += sum4(32 + lane);
      if (wv == 2 && gbase >= 0 && lane < nrows) acc[gbase + lane] += sum4(64 + lane);
      if (wv == 3 && gbase >= 0 && lane < nrows) acc[bbase + lane] += sum4(96 + lane);
    } else if (wv == 0 && lane == 32) {
      acc[scbase] += sum4(128);
    }
    __syncthreads();
  }
  // Up to two vectors of 32 row sums (a at abase + m, b at bbase + m for m < nrows) and one scalar.
  __device__ void rows(float* acc, float a, int abase, float b, int bbase, int nrows, float sc, int scbase) const {
    float* S = mine();
    if (lane < 32) {
      S[lane] = a;
      S[32 + lane] = b;
    }
    if (lane == 0) S[64] = sc;
    __syncthreads();
    if (wv == 0 && lane < nrows) {
      if (abase >= 0) acc[abase + lane] += sum4(lane);
      if (bbase >= 0) acc[bbase + lane] += sum4(32 + lane);
    }
    if (wv == 0 && lane == 0 && scbase >= 0) acc[scbase] += sum4(64);
    __syncthreads();
  }
};

// Output activation: 0 mu_max * sigmoid(y), 1 identity, 2 softplus (beta 1, threshold 20).
__device__ __forceinline__ float act_fwd(int act, float mu_max, float y) {
  if (act == 1) return y;
  if (act == 2) return y > 20.0f ? y : log1pf(expf(y));
  return mu_max / (1.0f + expf(-y));
}

__device__ __forceinline__ float act_grad(int act, float mu_max, float y) {
  if (act == 1) return 1.0f;
  if (act == 2 && y > 20.0f) return 1.0f;   // softplus above its threshold is y itself
  const float s = 1.0f / (1.0f + expf(-y));
  if (act == 2) return s;
  return mu_max * s * (1.0f - s);
}

// Position of point p for the three point sources.
__device__ __forceinline__ void point_position(const FwdArgs& a, int64_t p, bool valid, int64_t ray,
                                               int i, const RayRec& rr, float x[3]) {
  x[0] = x[1] = x[2] = 0.0f;
  if (!valid) return;
  if (a.mode == kModeRays) {
    if (rr.hit) {
      const float u = a.jitter ? a.jitter[ray * a.N + i] : jitter(a.seed, a.step, (uint32_t)ray, (uint32_t)i);
      sample_pos(a.geo, rr, i, u, x);
    }
  } else if (a.mode == kModePoints || (a.mode == kModeVoxelLoss && a.xn)) {
    x[0] = a.xn[3 * p];
    x[1] = a.xn[3 * p + 1];
    x[2] = a.xn[3 * p + 2];
  } else if (a.mode == kModeVoxelLoss) {
    voxel_point(a.seed, a.step, (uint32_t)p, x);
  } else {
    const int64_t nxy = (int64_t)a.dims[0] * a.dims[1];
    const int iz = (int)(p / nxy);
    const int64_t rem = p - (int64_t)iz * nxy;
    const int iy = (int)(rem / a.dims[0]);
    const int ix = (int)(rem - (int64_t)iy * a.dims[0]);
    x[0] = voxel_coord(ix, a.dims[0]);
    x[1] = voxel_coord(iy, a.dims[1]);
    x[2] = voxel_coord(iz, a.dims[2]);
  }
}

// MLP forward of one point (hidden activations kept for the backward pass).
template <int C, int W, int D, int P>
__device__ __forceinline__ void mlp_forward(const float* sp, const float* z, float (&hb)[D][W / 2], int lane) {
  using Ly = Lay<C, W, D, P>;
  if constexpr (P == 0) {
    layer_fwd<C, W>(sp + Ly::sW(0), sp + Ly::sb(0), z, hb[0], lane);
#pragma unroll
    for (int k = 1; k < D; ++k) layer_fwd<W, W>(sp + Ly::sW(k), sp + Ly::sb(k), hb[k - 1], hb[k], lane);
  } else {
    const bf16x8* w16 = reinterpret_cast<const bf16x8*>(sp);
    layer_fwd_bf16<C, W>(w16 + Ly::wf(0), sp + Ly::sb(0), z, hb[0], lane);
#pragma unroll
    for (int k = 1; k < D; ++k) layer_fwd_bf16<W, W>(w16 + Ly::wf(k), sp + Ly::sb(k), hb[k - 1], hb[k], lane);
  }
}

// Record offsets, step 1, for bin b (one 256-thread block; every thread calls it): exclusive scan of
// the bin's per-block counts -> offsets relative to the bin's first record; the bin's total.  part:
// 4 words of LDS.
__device__ void bin_row_scan(int b, const uint32_t* __restrict__ counts, int grid, uint32_t* __restrict__ rel,
                             uint32_t* __restrict__ totals, const uint32_t* __restrict__ edge,
                             const int32_t* __restrict__ edge_beg, const int32_t* __restrict__ edge_src,
                             uint32_t* part) {
  const int t = threadIdx.x;
  const int per = (grid + 255) / 256;
  const int w0 = t * per, w1 = min(grid, w0 + per);
  const uint32_t* row = counts + (size_t)b * grid;
  const int e0 = edge ? edge_beg[b] : 0, e1 = edge ? edge_beg[b + 1] : 0;
  auto count = [&](int w) -> uint32_t {   // a bin at a level boundary: the levels' edge rows
    if (e0 == e1) return row[w];
    uint32_t v = 0u;
    for (int k = e0; k < e1; ++k) v += edge[(size_t)edge_src[k] * grid + w];
    return v;
  };
  uint32_t s = 0;
  for (int w = w0; w < w1; ++w) s += count(w);
  // inclusive scan within the wave, then the four waves' totals through LDS
  const int lane = t & 63, wv = t >> 6;
  uint32_t inc = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(inc, o, 64);
    if (lane >= o) inc += v;
  }
  if (lane == 63) part[wv] = inc;
  __syncthreads();
  uint32_t before = 0u, total = 0u;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t v = part[q];
    before += q < wv ? v : 0u;
    total += v;
  }
  uint32_t run = before + inc - s;
  for (int w = w0; w < w1; ++w) {
    rel[(size_t)b * grid + w] = run;
    run += count(w);
  }
  if (t == 0) totals[b] = total;
  __syncthreads();   // part is written again by the next call
}

// ---------------------------------------------------------------------------------------------
// Forward kernel
// ---------------------------------------------------------------------------------------------
// PRE: rays mode with the encoding already stored by k_enc (a.enc_pre); only the network runs.
template <int L, int W, int D, int P, bool PRE>
__global__ void __launch_bounds__(kBlock, W == 32 ? 2 : 1) k_fwd(const FwdArgs a) {
  constexpr int C = 2 * L, RC = C / 2, RW = W / 2;
  using Ly = Lay<C, W, D, P>;
  extern __shared__ float smem[];
  float* sp = smem;
  uint32_t* hist = (!PRE && a.bin_counts) ? reinterpret_cast<uint32_t*>(smem + Ly::s_n) : nullptr;
  stage_params<C, W, D, P>(a.dense, sp);
  if (hist)
    for (int b2 = threadIdx.x; b2 < a.n_bins; b2 += blockDim.x) hist[b2] = 0u;
  __syncthreads();
  if constexpr (PRE) {   // the record offsets' row scans of the encoder's counts, bins spread over the grid
    __shared__ uint32_t part[kBlock / 64];
    if (a.scan_rel)
      for (int b2 = blockIdx.x; b2 < a.n_bins; b2 += gridDim.x)
        bin_row_scan(b2, a.scan_counts, a.enc_grid, a.scan_rel, a.scan_totals, a.edge_counts, a.edge_beg,
                     a.edge_src, part);
  }

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, n = lane & 31, h = lane >> 5;
  const int64_t n_chunks = (a.n_points + kPtsPerBlock - 1) / kPtsPerBlock;
  for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
    const int64_t wave_id = chunk * kWavesPerBlock + wv;
    const int64_t p = wave_id * kPtsPerWave + n;
    const bool wave_valid = wave_id * kPtsPerWave < a.n_points;
    const bool valid = p < a.n_points;
    int64_t ray = 0;
    int i = 0;
    RayRec rr{};
    if ((PRE || a.mode == kModeRays) && wave_valid) {
      ray = (wave_id * kPtsPerWave) / a.N;
      i = (int)(p - ray * a.N);
      rr = a.rays[ray];
    }
    const bool vloss = !PRE && a.mode == kModeVoxelLoss;

    float e[RC];
    if constexpr (PRE) {             // encoding computed by k_enc in this layout
#pragma unroll
      for (int r = 0; r < RC; ++r) e[r] = wave_valid ? a.enc_pre[(wave_id * RC + r) * kWave + lane] : 0.0f;
    } else if (a.mode == kModeFeatures) {   // given encoder outputs: register r of half h is channel chan(r, h)
#pragma unroll
      for (int r = 0; r < RC; ++r) e[r] = valid ? a.feats[p * C + chan(r, h)] : 0.0f;
    } else {
      float x[3];
      point_position(a, p, valid, ray, i, rr, x);
      const uint32_t tbase = vloss ? (uint32_t)(p / a.pts_per_table) * a.table_stride : 0u;
      // the bin histogram counts exactly the records the backward pass writes (hit rays only)
      encode_half<L, P>(a.lt, a.table, x, h, e, hist != nullptr, (valid && (rr.hit || vloss)) ? hist : nullptr,
                        n, tbase);
    }
    if (!PRE && a.enc_out && wave_valid) {
#pragma unroll
      for (int r = 0; r < RC; ++r) a.enc_out[(wave_id * RC + r) * kWave + lane] = e[r];
    }
    if (a.mask) {   // channel mask (Sec. 2.3) between the encoder and LayerNorm
#pragma unroll
      for (int r = 0; r < RC; ++r) e[r] *= a.mask[chan(r, h)];
    }
    float xh[RC], z[RC], rstd;
    ln_forward<C>(e, sp + Ly::s_lng, sp + Ly::s_lnb, a.ln_eps, a.layernorm, h, xh, z, rstd);

    float hb[D][RW];
    mlp_forward<C, W, D, P>(sp, z, hb, lane);
    float yp = 0.0f;
#pragma unroll
    for (int R = 0; R < RW; ++R) yp += sp[Ly::s_wo + chan(R, h)] * hb[D - 1][R];
    const float y = yp + xor32(yp) + sp[Ly::s_bo];
    const float mu = act_fwd(a.out_act, a.mu_max, y);

    if (PRE || a.mode == kModeRays) {
      float c = (h == 0 && valid) ? mu * rr.delta : 0.0f;
      c = half_sum(c);
      if (lane == 0 && wave_valid) a.wave_sum[wave_id] = c;
    } else if (!vloss && h == 0 && valid) {
      a.mu_out[p] = mu;
    }
  }
  if (hist) {
    __syncthreads();
    for (int b2 = threadIdx.x; b2 < a.n_bins; b2 += blockDim.x)
      a.bin_counts[(size_t)b2 * gridDim.x + blockIdx.x] = hist[b2];
  }
}

// ---------------------------------------------------------------------------------------------
// Level-major encoder of the ray training step
// ---------------------------------------------------------------------------------------------
// Block (l, w) computes level l of the hash encoding (Sec. 2.2) at the points of backward block w
// (chunks w, w + G, w + 2G, ... of kPtsPerBlock points, G = a.enc_grid), stores it where k_fwd and
// k_bwd read it (register 4(l/4) + 2(l%2) + f of lane half (l/2)%2, as encode_half leaves it) and
// counts the records block w of k_bwd will write for level l, per bin.
// Placement: workgroups go to the 8 XCDs of the chip in turn (block b to XCD b mod 8), so with
// b = 8 (phase * G + w) + x each XCD works on one level at a time, and that level's table (4 MB at
// FP32, 2 MB at FP16 for T = 2^19) stays in the XCD's own L2 instead of the whole table streaming
// through every L2.  The phases run over the levels in serpentine order (phase 0: l = x, phase 1:
// l = 15 - x, ...): a level costs more the finer it is, so each XCD pairs a coarse level with a
// fine one and the XCDs finish together.
// One lane per point; lanes 32k .. 32k + 31 of a wave hold the 32 points of one backward wave, so
// the runs (run_flags) and the records counted are exactly those of scatter_half.  Level l is
// skipped (zero encoding, no records) exactly when scatter_half and encode_half skip its pair.
// Counts: a bin strictly inside level l's entry range belongs to level l alone and its count is
// stored at bin_counts[bin][w]; the level's first and last bins, which other levels can share, go
// to edge_counts[2l][w] and edge_counts[2l + 1][w] (0 there when both are one bin), summed by
// the bin scan.
template <int L, int P>
__global__ void __launch_bounds__(kEncThreads) k_enc(const FwdArgs a) {
  constexpr int RC = L;   // channel registers per lane in the backward layout (C / 2)
  extern __shared__ float smem[];
  uint32_t* hist = reinterpret_cast<uint32_t*>(smem);
  const int G = a.enc_grid;
  const int s = (int)(blockIdx.x >> 3);
  const int ph = s / G, w = s - ph * G;
  const int x = (int)(blockIdx.x & 7u);
  const int l = 8 * ph + ((ph & 1) ? 7 - x : x);
  if (l >= L) return;                                   // block-uniform, before any barrier
  const LevelTab& T = a.lt;
  const int32_t N = T.res[l];
  const uint32_t off = T.off[l], st = T.stride[l];
  const uint32_t size = st ? st * st * st : T.mask + 1u;
  const uint32_t b0 = off >> T.bin_shift, b1 = (off + size - 1u) >> T.bin_shift;
  const int nbl = (int)(b1 - b0) + 1;
  const bool on = ((T.on >> l) | (T.on >> (l ^ 2))) & 1u;
  for (int k = threadIdx.x; k < nbl; k += blockDim.x) hist[k] = 0u;
  __syncthreads();

  const int t = threadIdx.x, ln = t & 31;
  const int hh = (l >> 1) & 1, r0 = 4 * (l >> 2) + 2 * (l & 1);
  const int64_t n_chunks = (a.n_points + kPtsPerBlock - 1) / kPtsPerBlock;
  constexpr int kChunksAtOnce = kEncThreads / kPtsPerBlock;
  for (int64_t c = w + (int64_t)(t / kPtsPerBlock) * G; c < n_chunks; c += (int64_t)kChunksAtOnce * G) {
    const int64_t p = c * kPtsPerBlock + (t % kPtsPerBlock);
    const bool valid = p < a.n_points;
    int64_t ray = 0;
    int i = 0;
    RayRec rr{};
    if (valid) {
      ray = p / a.N;
      i = (int)(p - ray * a.N);
      rr = a.rays[ray];
    }
    float x[3];
    point_position(a, p, valid, ray, i, rr, x);
    float s0 = 0.0f, s1 = 0.0f;
    if (on) {
      uint32_t idx[8];
      float wt[8];
      uint32_t g0, g1, g2;
      level_corners(N, off, st, T.mask, x, idx, wt, g0, g1, g2);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        float2 v;
        if constexpr (P == 0) v = reinterpret_cast<const float2*>(a.table)[idx[k]];
        else v = __half22float2(reinterpret_cast<const __half2*>(a.table)[idx[k]]);
        s0 += wt[k] * v.x;
        s1 += wt[k] * v.y;
      }
      bool cont, tail;
      run_flags(g0, g1, g2, ln, cont, tail);
      if (valid && rr.hit && tail) {
#pragma unroll
        for (int k = 0; k < 8; ++k) atomicAdd(hist + ((idx[k] >> T.bin_shift) - b0), 1u);
      }
    }
    // Stored non-temporally: each half-wave writes one whole 128-B line per channel, and keeping
    // the encoding out of the L2 leaves the L2 to the level's table.
    const int64_t wid = p / kPtsPerWave;
    if (wid * kPtsPerWave < a.n_points) {
      float* dst = a.enc_out + (wid * RC + r0) * kWave + ln + 32 * hh;
      __builtin_nontemporal_store(s0, dst);
      __builtin_nontemporal_store(s1, dst + kWave);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nbl; k += blockDim.x) {
    const uint32_t v = hist[k];
    if (k == 0) a.edge_counts[(size_t)(2 * l) * G + w] = v;
    else if (k == nbl - 1) a.edge_counts[(size_t)(2 * l + 1) * G + w] = v;
    else a.bin_counts[(size_t)(b0 + k) * G + w] = v;
  }
  if (nbl == 1 && threadIdx.x == 0) a.edge_counts[(size_t)(2 * l + 1) * G + w] = 0u;
}

// ---------------------------------------------------------------------------------------------
// Backward kernel (persistent over 128-point chunks)
// ---------------------------------------------------------------------------------------------
// Floats of k_bwd's LDS after the staged parameters and before the bin cursors: W = 32 the dense
// accumulator and two tiles per wave; W = 64 four tile slots per wave, which the dense gradient
// reuses at the end.
template <int W>
__host__ __device__ constexpr int bwd_tiles_lds(int nd_pad) {
  return W == 64 ? (nd_pad > 4 * kWavesPerBlock * 32 * kTile ? nd_pad : 4 * kWavesPerBlock * 32 * kTile)
                 : nd_pad + kWavesPerBlock * 2 * 32 * kTile;
}

template <int L, int W, int D, int P>
__global__ void __launch_bounds__(kBlock, W == 32 ? 2 : 1) k_bwd(const FwdArgs a, const BwdArgs b) {
  constexpr int C = 2 * L, RC = C / 2, RW = W / 2;
  using Ly = Lay<C, W, D, P>;
  // 64 wide (one block per CU): every wave owns one 32x32 weight-gradient tile of each layer and
  // sums it in registers over all 128 points of every chunk, reading the other waves' blocks from
  // four tile slots per wave; the block's dense gradient is assembled once, at the end.  32 wide:
  // each wave's tiles over its own 32 points, combined across the waves chunk by chunk.
  constexpr bool kOwn = W == 64;
  constexpr int kSlot = 32 * kTile, nd_pad = (Ly::g_n + 3) & ~3;
  extern __shared__ float smem[];
  float* sp = smem;
  float* acc = smem + Ly::s_n;                  // kOwn: assembled at the end, over the slots
  float* const slots = smem + Ly::s_n;          // kOwn: slots [wave][4][32][kTile]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, n = lane & 31, h = lane >> 5;
  float* tG = kOwn ? slots + (4 * wv + 3) * kSlot : acc + nd_pad + wv * (2 * kSlot);
  float* tH = tG + kSlot;                       // (not used when kOwn)
  uint32_t* cursor = reinterpret_cast<uint32_t*>(smem + Ly::s_n + bwd_tiles_lds<W>(nd_pad));

  stage_params<C, W, D, P>(a.dense, sp);
  if constexpr (!kOwn)
    for (int e2 = threadIdx.x; e2 < nd_pad; e2 += blockDim.x) acc[e2] = 0.0f;
  for (int b2 = threadIdx.x; b2 < a.n_bins; b2 += blockDim.x)
    cursor[b2] = b.bin_start[b2] + b.bin_offsets[(size_t)b2 * gridDim.x + blockIdx.x];
  __syncthreads();

  const int waves_per_ray = a.N / kPtsPerWave;
  const int64_t n_chunks = (a.n_points + kPtsPerBlock - 1) / kPtsPerBlock;
  uint32_t vbits = 0u;   // largest |record| as a bit pattern: NaN and inf order above every finite value
  bool bad = false;      // a residual, upstream gradient or dense partial that is not finite
  // kOwn: the wave's weight-gradient tile of each layer, and its own points' bias, output-unit and
  // LayerNorm row sums (row lane % 32), over the block's chunks
  f32x16 ownW[D];
  float ownB[D][2], ownWo[2] = {0.0f, 0.0f}, ownLg = 0.0f, ownLb = 0.0f, ownBo = 0.0f;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    ownW[k] = f32x16{};
    ownB[k][0] = ownB[k][1] = 0.0f;
  }
  for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
    const int64_t wave_id = chunk * kWavesPerBlock + wv;
    const int64_t p = wave_id * kPtsPerWave + n;
    const bool wave_valid = wave_id * kPtsPerWave < a.n_points;
    const bool valid = p < a.n_points;
    int64_t ray = 0;
    int i = 0;
    RayRec rr{};
    const bool vloss = a.mode == kModeVoxelLoss;
    if (wave_valid && !vloss) {
      ray = (wave_id * kPtsPerWave) / a.N;
      i = (int)(p - ray * a.N);
      rr = a.rays[ray];
    }
    float x[3];
    point_position(a, p, valid, ray, i, rr, x);
    const uint32_t tid = vloss ? (uint32_t)(p / a.pts_per_table) : 0u;
    const uint32_t tbase = tid * a.table_stride;

    float e[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) e[r] = wave_valid ? b.enc_in[(wave_id * RC + r) * kWave + lane] : 0.0f;
    if (a.mask) {   // channel mask (Sec. 2.3) between the encoder and LayerNorm
#pragma unroll
      for (int r = 0; r < RC; ++r) e[r] *= a.mask[chan(r, h)];
    }
    float xh[RC], z[RC], rstd;
    ln_forward<C>(e, sp + Ly::s_lng, sp + Ly::s_lnb, a.ln_eps, a.layernorm, h, xh, z, rstd);

    float hb[D][RW];
    mlp_forward<C, W, D, P>(sp, z, hb, lane);
    float yp = 0.0f;
#pragma unroll
    for (int R = 0; R < RW; ++R) yp += sp[Ly::s_wo + chan(R, h)] * hb[D - 1][R];
    const float y = yp + xor32(yp) + sp[Ly::s_bo];

    // Upstream gradient of the ray sum (Eq. 3), or of the voxel loss (Eq. 2).
    float dA = 0.0f;
    float dmu_vox = 0.0f;
    if (vloss) {
      const float mu = act_fwd(a.out_act, a.mu_max, y);
      const float tgt = trilinear(a.vols + (size_t)tid * a.vol_n * a.vol_n * a.vol_n, a.vol_n, x);
      const float res = mu - tgt;
      bad |= valid && !(fabsf(res) <= FLT_MAX);
      dmu_vox = valid ? (float)((res > 0.0f) - (res < 0.0f)) * b.inv_R : 0.0f;
      const float l = half_sum((h == 0 && valid) ? fabsf(res) : 0.0f);
      if (lane == 0 && wave_valid) b.wave_loss[wave_id] = l;
    } else if (wave_valid) {
      if (b.dA_in) {
        dA = b.dA_in[ray];
        bad |= !(fabsf(dA) <= FLT_MAX);
      } else {
        float A = 0.0f;
        for (int w2 = 0; w2 < waves_per_ray; ++w2) A += a.wave_sum[ray * waves_per_ray + w2];
        const float res = A - rr.a_gt;
        bad |= !(fabsf(res) <= FLT_MAX);
        dA = (float)((res > 0.0f) - (res < 0.0f)) * b.inv_R;
        if (i == 0 && lane == 0) {
          if (b.a_pred_out) b.a_pred_out[ray] = A;
          if (b.absres_out) b.absres_out[ray] = fabsf(res);
        }
      }
    }
    const float dmu = vloss ? dmu_vox : ((valid && rr.hit) ? dA * rr.delta : 0.0f);
    const float dy = dmu * act_grad(a.out_act, a.mu_max, y);

    // Output unit.
    float g[RW];
    float t[RW];
#pragma unroll
    for (int R = 0; R < RW; ++R) {
      g[R] = dy * sp[Ly::s_wo + chan(R, h)];
      t[R] = dy * hb[D - 1][R];
    }
    const Combine cmb{acc + nd_pad, 2 * 32 * kTile, wv, lane};
    const float sdy = half_sum(h == 0 ? dy : 0.0f);
    // row sums of the output weights' gradient (kOwn: in slot 3, which no other wave reads from
    // the last layer's outer products of a chunk to the first one's of the next), combined across
    // waves with the LayerNorm's below
    float rs[W / 32];
#pragma unroll
    for (int mb = 0; mb < W / 32; ++mb) {
      tile_put<RW>(tG, t, mb, lane);
      wave_lds_sync();
      rs[mb] = tile_rowsum(tG, lane);
      wave_lds_sync();
    }
    if constexpr (kOwn) {
      ownWo[0] += rs[0];
      ownWo[1] += rs[W / 32 - 1];
      ownBo += sdy;
    }

    // Hidden layers, last to first.  Weight gradients: per 32x32 block, the FP32 tile of the layer's
    // output gradient gives the bias row sums; the outer product over the wave's 32 points runs on
    // MFMA (FP32 tiles, or bf16 tiles overlaid on the consumed FP32 ones in the BF16 form).
    float gz[RC];
    __bf16* tGb = reinterpret_cast<__bf16*>(tH);
    __bf16* tHb = reinterpret_cast<__bf16*>(tG);
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
      float ga[RW];
#pragma unroll
      for (int R = 0; R < RW; ++R) ga[R] = hb[k][R] > 0.0f ? g[R] : 0.0f;
      const int Kk = Ly::K(k);
      const float* hin = (k == 0) ? z : hb[k > 0 ? k - 1 : 0];
      if constexpr (kOwn) {
        // slots 0, 1: the wave's output-gradient blocks (FP32 for its bias row sums, then the
        // BF16 operand tiles in the BF16 form); slots 2, 3: its input blocks (one at layer 0)
        float* S = slots + 4 * wv * kSlot;
        __syncthreads();                        // every wave is done with the slots' last contents
        tile_put<RW>(S, ga, 0, lane);
        tile_put<RW>(S + kSlot, ga, 1, lane);
        wave_lds_sync();
        ownB[k][0] += tile_rowsum(S, lane);
        ownB[k][1] += tile_rowsum(S + kSlot, lane);
        if constexpr (P == 1) {
          wave_lds_sync();
          tile_put_bf16<RW>(reinterpret_cast<__bf16*>(S), ga, 0, lane);
          tile_put_bf16<RW>(reinterpret_cast<__bf16*>(S + kSlot), ga, 1, lane);
        }
        if (k == 0) {
          if constexpr (P == 0) tile_put<RC>(S + 2 * kSlot, z, 0, lane);
          else tile_put_bf16<RC>(reinterpret_cast<__bf16*>(S + 2 * kSlot), z, 0, lane);
        } else {
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            if constexpr (P == 0) tile_put<RW>(S + (2 + nb) * kSlot, hin, nb, lane);
            else tile_put_bf16<RW>(reinterpret_cast<__bf16*>(S + (2 + nb) * kSlot), hin, nb, lane);
          }
        }
        __syncthreads();                        // every wave's blocks are in place
        // the wave's tile: hidden layers (mb, nb) = (wv / 2, wv % 2) over the chunk's 128 points;
        // layer 0 (one input block) rows mb = wv % 2 over the points of waves 2 (wv / 2) and + 1
        const int mb = k == 0 ? (wv & 1) : (wv >> 1), nb = k == 0 ? 0 : (wv & 1);
        const int q0 = k == 0 ? 2 * (wv >> 1) : 0;
#pragma unroll
        for (int q = 0; q < (k == 0 ? 2 : kWavesPerBlock); ++q) {
          const float* Sq = slots + 4 * (q0 + q) * kSlot;
          if constexpr (P == 0) ownW[k] = tile_outer(Sq + mb * kSlot, Sq + (2 + nb) * kSlot, lane, ownW[k]);
          else
            ownW[k] = tile_outer_bf16(reinterpret_cast<const __bf16*>(Sq + mb * kSlot),
                                      reinterpret_cast<const __bf16*>(Sq + (2 + nb) * kSlot), lane, ownW[k]);
        }
      } else {
#pragma unroll
      for (int mb = 0; mb < W / 32; ++mb) {
        tile_put<RW>(tG, ga, mb, lane);
        if constexpr (P == 1) tile_put_bf16<RW>(tGb, ga, mb, lane);
        wave_lds_sync();
        const float brow = tile_rowsum(tG, lane);
        wave_lds_sync();
#pragma unroll
        for (int nb = 0; nb < (Kk + 31) / 32; ++nb) {
          f32x16 d;
          if constexpr (P == 0) {
            if (k == 0) tile_put<RC>(tH, z, nb, lane);
            else tile_put<RW>(tH, hin, nb, lane);
            wave_lds_sync();
            d = tile_outer(tG, tH, lane);
          } else {
            if (k == 0) tile_put_bf16<RC>(tHb, z, nb, lane);
            else tile_put_bf16<RW>(tHb, hin, nb, lane);
            wave_lds_sync();
            d = tile_outer_bf16(tGb, tHb, lane);
          }
          wave_lds_sync();
          // stage in the slot whose tile is no longer needed: tH (FP32 form) / tG (BF16 form)
          const Combine c2{P == 0 ? acc + nd_pad + 32 * kTile : acc + nd_pad, 2 * 32 * kTile, wv, lane};
          c2.tile(acc, d, Ly::gW(k), Kk, mb, nb, brow, nb == 0 ? Ly::gb(k) : -1);
        }
      }
      }
      if (k > 0) {
        float gp[RW];
        if constexpr (P == 0) layer_bwd_data<W, W>(sp + Ly::sW(k), ga, gp, lane);
        else layer_bwd_data_bf16<W, W>(reinterpret_cast<const bf16x8*>(sp) + Ly::wb(k), ga, gp, lane);
#pragma unroll
        for (int R = 0; R < RW; ++R) g[R] = gp[R];
      } else {
        if constexpr (P == 0) layer_bwd_data<C, W>(sp + Ly::sW(0), ga, gz, lane);
        else layer_bwd_data_bf16<C, W>(reinterpret_cast<const bf16x8*>(sp) + Ly::wb(0), ga, gz, lane);
      }
    }

    // LayerNorm backward.
    float gx[RC];
    if (a.layernorm) {
      float t1[RC], t2[RC];
      float sg = 0.0f, sgx = 0.0f;
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        t1[r] = gz[r] * xh[r];
        t2[r] = gz[r];
        const float gg = sp[Ly::s_lng + chan(r, h)] * gz[r];
        sg += gg;
        sgx += gg * xh[r];
      }
      if constexpr (kOwn) {   // slot 3 only (the other slots may still be read by layer 0's tiles)
        tile_put<RC>(tG, t1, 0, lane);
        wave_lds_sync();
        ownLg += tile_rowsum(tG, lane);
        wave_lds_sync();
        tile_put<RC>(tG, t2, 0, lane);
        wave_lds_sync();
        ownLb += tile_rowsum(tG, lane);
        wave_lds_sync();
      } else {
        tile_put<RC>(tG, t1, 0, lane);
        tile_put<RC>(tH, t2, 0, lane);
        wave_lds_sync();
        const float rg = tile_rowsum(tG, lane), rb = tile_rowsum(tH, lane);
        wave_lds_sync();
        cmb.rows_merged(acc, rs[0], rs[W / 32 - 1], W == 64, Ly::g_wo, rg, rb, Ly::g_lng, Ly::g_lnb, C, sdy,
                        Ly::g_bo);
      }
      sg += xor32(sg);
      sgx += xor32(sgx);
      const float mg = sg * (1.0f / C), mgx = sgx * (1.0f / C);
#pragma unroll
      for (int r = 0; r < RC; ++r)
        gx[r] = rstd * (sp[Ly::s_lng + chan(r, h)] * gz[r] - mg - xh[r] * mgx);
    } else {
      if constexpr (!kOwn)
        cmb.rows_merged(acc, rs[0], rs[W / 32 - 1], W == 64, Ly::g_wo, 0.0f, 0.0f, -1, -1, 0, sdy, Ly::g_bo);
#pragma unroll
      for (int r = 0; r < RC; ++r) gx[r] = gz[r];
    }

    if (a.mask) {   // back through the channel mask to the raw encoding
#pragma unroll
      for (int r = 0; r < RC; ++r) gx[r] *= a.mask[chan(r, h)];
    }
    scatter_half<L>(a.lt, b.recs, cursor, x, h, gx, valid && (rr.hit || vloss), n, tbase, b.rec_cap, vbits);
  }
  // Largest |record| of the step (non-negative floats order like their bit patterns): sets the
  // fixed-point scale of the bin reduction.
  for (int o = 32; o >= 1; o >>= 1) vbits = max(vbits, (uint32_t)__shfl_xor((int)vbits, o, 64));
  if (lane == 0) atomicMax(b.rec_max_bits, vbits);
  bad |= vbits >= 0x7F800000u;

  if constexpr (kOwn) {   // the block's dense gradient from the waves' registers, in a fixed order
    __syncthreads();                            // the slots are free
    for (int e2 = threadIdx.x; e2 < nd_pad; e2 += blockDim.x) acc[e2] = 0.0f;
    __syncthreads();
    const int m = lane & 31;
#pragma unroll
    for (int k = 1; k < D; ++k) {               // hidden layers: each tile has one owner
      const int mb = wv >> 1, nb = wv & 1;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[Ly::gW(k) + (32 * mb + chan(r, h)) * W + 32 * nb + m] = ownW[k][r];
    }
    for (int pass = 0; pass < 2; ++pass) {      // layer 0: waves 0, 1, then 2, 3 add their halves
      if ((wv >> 1) == pass && m < C) {
        const int mb = wv & 1;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[Ly::gW(0) + (32 * mb + chan(r, h)) * C + m] += ownW[0][r];
      }
      __syncthreads();
    }
    for (int q = 0; q < kWavesPerBlock; ++q) {  // the row sums, wave by wave
      if (wv == q && lane < 32) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
          acc[Ly::gb(k) + lane] += ownB[k][0];
          acc[Ly::gb(k) + 32 + lane] += ownB[k][1];
        }
        acc[Ly::g_wo + lane] += ownWo[0];
        acc[Ly::g_wo + 32 + lane] += ownWo[1];
        if (a.layernorm && lane < C) {
          acc[Ly::g_lng + lane] += ownLg;
          acc[Ly::g_lnb + lane] += ownLb;
        }
        if (lane == 0) acc[Ly::g_bo] += ownBo;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int e2 = threadIdx.x; e2 < nd_pad; e2 += blockDim.x) {
    const float v = acc[e2];
    bad |= !(fabsf(v) <= FLT_MAX);
    b.partials[(size_t)blockIdx.x * nd_pad + e2] = v;
  }
  // A non-finite value anywhere in the step: the reductions write nothing from here on (this step
  // and every later one) until the host reads the flag and clears it.
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicCAS(b.bad_step, 0u, a.step + 1u);
}

// ---------------------------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------------------------
// Ray r of a batch: pixel (given or drawn), FP64 set-up, measured line integral.
__device__ __forceinline__ void ray_one(const RaysArgs& a, int r) {
  const int32_t pix = a.pix_in ? a.pix_in[r] : draw_pixel(a.seed, a.step, a.h_bits, a.n_pix, (uint32_t)r);
  RayRec rec;
  const bool in_range = pix >= 0 && (uint32_t)pix < a.n_pix;
  ray_setup(a.geo, a.ca, a.sa, in_range ? pix : 0, a.N, rec);
  if (!in_range) {            // a pixel index outside the detector is a ray that misses
    rec.hit = 0;
    rec.delta = 0.0f;
    rec.pix = pix;
  }
  rec.a_gt = (a.proj && in_range) ? a.proj[(size_t)a.view * a.n_pix + pix] : 0.0f;
  a.rays[r] = rec;
  if (a.pix_out) a.pix_out[r] = pix;
  if (a.jitter_out)
    for (int i = 0; i < a.N; ++i) a.jitter_out[(size_t)r * a.N + i] = jitter(a.seed, a.step, (uint32_t)r, (uint32_t)i);
}

__global__ void k_rays(const RaysArgs a) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < a.n_rays) ray_one(a, r);
}

// A_pred of each ray from the per-wave partial sums (fixed order).
__global__ void k_raysum(const float* __restrict__ wave_sum, int waves_per_ray, int n_rays,
                         float* __restrict__ a_pred) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  float A = 0.0f;
  for (int w = 0; w < waves_per_ray; ++w) A += wave_sum[(size_t)r * waves_per_ray + w];
  a_pred[r] = A;
}

// Dense (LayerNorm + MLP) gradient, one 1024-thread block per 64 parameters (block index blk):
// grad_dense[k] += sum_g partials[g][k] (fixed order: 16 strided groups, then the groups in order);
// block 0 also forms loss = sum_r absres[r] * inv_R.  With fused != 0 the summed gradient goes into
// Adam on the dense parameters p/m/v instead and grad_dense is left at zero.  Runs as the last
// blocks of k_bin_combine (it only needs k_bwd's partials).
__device__ void dense_reduce_block(const DenseReduceArgs& d, int blk, float* red) {
  const int k = blk * 64 + (threadIdx.x & 63);
  const int grp = threadIdx.x >> 6;
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  if (k < d.nd) {
    int gi = grp;
    for (; gi + 48 < d.n_blocks; gi += 64) {
      s0 += d.partials[(size_t)gi * d.nd_pad + k];
      s1 += d.partials[(size_t)(gi + 16) * d.nd_pad + k];
      s2 += d.partials[(size_t)(gi + 32) * d.nd_pad + k];
      s3 += d.partials[(size_t)(gi + 48) * d.nd_pad + k];
    }
    for (; gi < d.n_blocks; gi += 16) s0 += d.partials[(size_t)gi * d.nd_pad + k];
  }
  red[threadIdx.x] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (grp == 0 && k < d.nd && *d.bad_step == 0u) {
    float t = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[threadIdx.x + 64 * q];
    if (d.fused) {
      float pp = d.p[k], mm = d.m[k], vv = d.v[k];
      adam_update(pp, mm, vv, d.grad_dense[k] + t, d.adam);
      d.p[k] = pp;
      d.m[k] = mm;
      d.v[k] = vv;
      d.grad_dense[k] = 0.0f;
    } else {
      d.grad_dense[k] += t;
    }
  }
  if (blk == 0 && d.loss_out) {
    __syncthreads();
    float l = 0.0f;
    for (int r = threadIdx.x; r < d.n_rays; r += blockDim.x) l += d.absres[r];
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) *d.loss_out = red[0] * d.inv_R;
  }
}

// Adam (Kingma and Ba, Algorithm 1) over float4 groups; resets the gradient; refreshes the FP16
// table copy when present.  n4 = number of float4 groups; the table occupies the first n_table
// floats.
__global__ void k_adam(float4* __restrict__ p, float4* __restrict__ g, float4* __restrict__ m,
                       float4* __restrict__ v, int64_t n4, float lr, float b1, float b2, float eps,
                       float ibc1, float ibc2, __half* __restrict__ th, int64_t n_table,
                       const uint32_t* __restrict__ bad_step) {
  if (*bad_step) return;   // a non-finite value was met: the model is left as it is
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += stride) {
    float4 pp = p[q], gg = g[q], mm = m[q], vv = v[q];
    float* P = &pp.x;
    float* G = &gg.x;
    float* M = &mm.x;
    float* V = &vv.x;
    const AdamArgs A{lr, b1, b2, eps, ibc1, ibc2};
#pragma unroll
    for (int k = 0; k < 4; ++k) adam_update(P[k], M[k], V[k], G[k], A);
    p[q] = pp;
    m[q] = mm;
    v[q] = vv;
    g[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (th && 4 * q < n_table) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (4 * q + k < n_table) th[4 * q + k] = __float2half_rn(P[k]);
    }
  }
}

// Count of the values of x that are NaN or infinite (grid-stride; one atomic per block).
__global__ void __launch_bounds__(256) k_count_nonfinite(const float* __restrict__ x, int64_t n,
                                                         uint32_t* __restrict__ count) {
  uint32_t c = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride)
    c += !(fabsf(x[q]) <= FLT_MAX);
  for (int o = 32; o >= 1; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o, 64);
  __shared__ uint32_t part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t t = part[0] + part[1] + part[2] + part[3];
    if (t) atomicAdd(count, t);
  }
}

__global__ void k_fill(float* __restrict__ x, int64_t n, float val) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) x[q] = val;
}

__global__ void k_to_half(const float* __restrict__ src, __half* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) dst[q] = __float2half_rn(src[q]);
}

// Initial values: table (2u - 1) 1e-4; linear layer weights and biases (2u - 1) / sqrt(fan_in);
// LayerNorm gain 1, bias 0.  u from Philox with counter (index, 0/hi, 0, stream).
__global__ void k_init(float* __restrict__ params, int64_t n_table, int64_t dense_off, InitArgs ia) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_table; q += stride) {
    const float u = u24f(philox_w0(ia.seed, (uint32_t)q, (uint32_t)((uint64_t)q >> 32), 0, kTable));
    params[q] = (2.0f * u - 1.0f) * 1e-4f;
  }
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ia.n_dense; k += stride) {
    float val;
    if (k < ia.ln_end) {
      val = (k < ia.ln_end / 2) ? 1.0f : 0.0f;
    } else {
      int fan = ia.width;
      if (k < ia.first_layer_end) fan = ia.fan0;
      const float u = u24f(philox_w0(ia.seed, (uint32_t)k, 0, 0, kMlp));
      val = (2.0f * u - 1.0f) / sqrtf((float)fan);
    }
    params[dense_off + k] = val;
  }
}

__global__ void __launch_bounds__(256) k_bin_rowscan(const uint32_t* __restrict__ counts, int grid,
                                                     uint32_t* __restrict__ rel, uint32_t* __restrict__ totals,
                                                     const uint32_t* __restrict__ edge,
                                                     const int32_t* __restrict__ edge_beg,
                                                     const int32_t* __restrict__ edge_src) {
  __shared__ uint32_t part[4];
  bin_row_scan(blockIdx.x, counts, grid, rel, totals, edge, edge_beg, edge_src, part);
}

// Record offsets, step 2 (one block): bin starts (exclusive scan of the bin totals, with the total T
// at index n_bins), and the ranges of the bin reduction's G' = min(G, T) blocks.  A block's time is its
// records plus a flush for every bin it ends, so the ranges split the cost (records + kFlushCost per
// non-empty bin, the flush counted at the bin's end) evenly: block j starts at the record where the
// cost reaches C j / G' (a boundary inside a bin's flush share falls on the bin's end).  Ranges may be
// empty.  block_first_bin[j]: the bin holding record block_start[j] (any bin when that is T).
__global__ void __launch_bounds__(1024) k_bin_plan(const uint32_t* __restrict__ totals, int n_bins, int G,
                                                   uint32_t* __restrict__ bin_start,
                                                   uint32_t* __restrict__ block_start,
                                                   int32_t* __restrict__ block_first_bin,
                                                   uint32_t* __restrict__ rec_max_bits) {
  if (threadIdx.x == 0) *rec_max_bits = 0u;
  constexpr int kWaves = 1024 / 64;
  __shared__ uint32_t part[kWaves];
  __shared__ unsigned long long cpart[kWaves];
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wv = t >> 6;
  const int per = (n_bins + nt - 1) / nt;
  const int b0 = t * per, b1 = min(n_bins, b0 + per);
  uint32_t srec = 0;
  unsigned long long scost = 0;
  for (int b = b0; b < b1; ++b) {
    const uint32_t tot = totals[b];
    srec += tot;
    scost += tot ? (unsigned long long)tot + kFlushCost : 0ull;
  }
  // inclusive scans within each wave, then the waves' totals through LDS
  uint32_t ir = srec;
  unsigned long long ic = scost;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t vr = __shfl_up(ir, o, 64);
    const unsigned long long vc = __shfl_up(ic, o, 64);
    if (lane >= o) {
      ir += vr;
      ic += vc;
    }
  }
  if (lane == 63) {
    part[wv] = ir;
    cpart[wv] = ic;
  }
  __syncthreads();
  uint64_t T = 0, C = 0;
  uint32_t rec = ir - srec;
  unsigned long long cst = ic - scost;
  for (int q = 0; q < nt / 64; ++q) {
    T += part[q];
    C += cpart[q];
    if (q < wv) {
      rec += part[q];
      cst += cpart[q];
    }
  }
  const uint64_t Ge = T < (uint64_t)G ? T : (uint64_t)G;
  for (int b = b0; b < b1; ++b) {
    const uint32_t tot = totals[b];
    bin_start[b] = rec;
    if (tot > 0) {   // blocks j whose cost boundary C j / G' lies in [cst, cst + tot + F)
      const unsigned long long c1 = cst + tot + kFlushCost;
      const uint64_t j0 = (cst * Ge + C - 1) / C, j1 = min((c1 * Ge + C - 1) / C, Ge);
      for (uint64_t j = j0; j < j1; ++j) {
        const uint64_t tj = C * j / Ge - cst;
        if (tj < tot) {
          block_start[j] = rec + (uint32_t)tj;
          block_first_bin[j] = b;
        } else {   // at the bin's end: the block starts in the next bin with records (or at T, empty)
          block_start[j] = rec + tot;
          int nb = b + 1;
          while (nb < n_bins && totals[nb] == 0) ++nb;
          block_first_bin[j] = nb < n_bins ? nb : n_bins - 1;
        }
      }
      cst = c1;
    }
    rec += tot;
  }
  if (t == nt - 1) {
    bin_start[n_bins] = (uint32_t)T;
    block_start[Ge] = (uint32_t)T;
  }
}

// Table gradient from the records.  Block j streams its share of the records (grouped by bin)
// and sums each bin's part in a 2^kBinBits-entry LDS tile (one pass over the part per tile when a
// bin spans several tiles).  The tile accumulates in int64 fixed point: LDS integer atomics are an
// order of magnitude faster than LDS float atomics on gfx950, and integer sums are exact, so the
// result does not depend on record order.  Scale 2^e per bin: with c records in the bin and every
// |record| <= vmax, |sum| <= c vmax < 2^61 2^-e, so no partial sum overflows; each record is rounded
// once to a multiple of 2^-e (error <= 2^-e-1 = c vmax 2^-63).
// A bin inside the block's range is added straight into the FP32 gradient (the block owns those
// entries), or, in a fused training step, handed to Adam on the entries' parameters and moments.  A
// bin cut by range boundaries is held by consecutive blocks j0..j1: each stores its int64 tile in
// its own slot (2j for its first bin, 2j+1 for its last) and k_bin_combine adds the slots in block
// order after the kernel ends (no cross-block synchronisation inside a kernel).  In a fused step
// k_bin_combine also runs Adam on the entries of bins without records.

// Moves the summed tile out (and leaves it zero): Adam on the entries (fused), added to the gradient,
// or, for a cut bin, stored as int64 in the block's slot.  Called by all threads after a barrier.
// The entries' parameters and moments (or gradient) are loaded here, not ahead of time: registers
// held across the record stream would cost the stream its second buffer, and the waves of the
// block still streaming their next chunk hide the latency.
template <bool FUSED>
__device__ __forceinline__ void tile_flush(const BinReduceArgs& a, unsigned long long* tile64, uint32_t base,
                                           int64_t lim, bool split, size_t slot, int sub, double down) {
  constexpr int NB = 1 << kBinBits;
  if (split) {
    unsigned long long* S = a.split_acc + (slot * a.n_sub + sub) * (2 * NB);
    for (int e2 = threadIdx.x; e2 < 2 * NB; e2 += kReduceThreads) {
      S[e2] = tile64[e2];
      tile64[e2] = 0ull;
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < kBinTilePer; ++k) {
    const int q = k * kReduceThreads + threadIdx.x;
    const long long s0 = (long long)tile64[2 * q], s1 = (long long)tile64[2 * q + 1];
    tile64[2 * q] = 0ull;
    tile64[2 * q + 1] = 0ull;
    if (q < lim) {
      const float d0 = (float)((double)s0 * down), d1 = (float)((double)s1 * down);
      if constexpr (FUSED) {
        float2 pp = reinterpret_cast<const float2*>(a.p)[base + q];
        float2 mm = reinterpret_cast<const float2*>(a.m)[base + q];
        float2 vv = reinterpret_cast<const float2*>(a.v)[base + q];
        adam_update(pp.x, mm.x, vv.x, d0, a.adam);
        adam_update(pp.y, mm.y, vv.y, d1, a.adam);
        reinterpret_cast<float2*>(a.p)[base + q] = pp;
        reinterpret_cast<float2*>(a.m)[base + q] = mm;
        reinterpret_cast<float2*>(a.v)[base + q] = vv;
        if (a.th) reinterpret_cast<__half2*>(a.th)[base + q] = __floats2half2_rn(pp.x, pp.y);
      } else {
        float2 o = reinterpret_cast<const float2*>(a.grad_table)[base + q];
        o.x += d0;
        o.y += d1;
        reinterpret_cast<float2*>(a.grad_table)[base + q] = o;
      }
    }
  }
}

__device__ __forceinline__ void rec_add(unsigned long long* tile64, const BinRec& r, uint32_t base, double up) {
  const uint32_t q = r.idx - base;   // wraps above NB for records of another tile
  if (q < (uint32_t)(1 << kBinBits)) {
    atomicAdd(tile64 + 2 * q, (unsigned long long)__double2ll_rn((double)r.v0 * up));
    atomicAdd(tile64 + 2 * q + 1, (unsigned long long)__double2ll_rn((double)r.v1 * up));
  }
}

template <bool FUSED>
__global__ void __launch_bounds__(kReduceThreads) k_bin_reduce(const BinReduceArgs a) {
  extern __shared__ unsigned long long tile64[];
  __shared__ uint32_t sb[65];                                      // bin starts of the block's first bins
  constexpr int NB = 1 << kBinBits;
  constexpr int U = 4, CH = U * kReduceThreads;                    // records per thread / block per chunk
  const uint64_t T = a.bin_start[a.n_bins];
  const uint64_t Ge = T < (uint64_t)gridDim.x ? T : (uint64_t)gridDim.x;
  const uint64_t jb = blockIdx.x;
  if (jb >= Ge) return;                                            // block-uniform
  if (*a.bad_step) return;                                         // non-finite step: write nothing
  const uint32_t rs = a.block_start[jb], re = a.block_start[jb + 1];
  if (rs >= re) return;                                            // an empty range
  const float vmax = __uint_as_float(*a.rec_max_bits);
  int ev;
  frexpf(vmax, &ev);                                               // vmax < 2^ev
  const int first_bin = a.block_first_bin[jb];
  if (threadIdx.x < 65 && first_bin + (int)threadIdx.x <= a.n_bins) sb[threadIdx.x] = a.bin_start[first_bin + threadIdx.x];
  for (int e2 = threadIdx.x; e2 < 2 * NB; e2 += kReduceThreads) tile64[e2] = 0ull;
  __syncthreads();
  auto bstart = [&](int B) -> uint32_t { return B - first_bin < 65 ? sb[B - first_bin] : a.bin_start[B]; };

  // current segment: the part of bin B inside [rs, re)
  int B = first_bin;
  uint32_t b_start = bstart(B), b_end = bstart(B + 1);
  uint32_t seg_end, base;
  int64_t lim;
  bool split;
  double up, down;
  auto begin_segment = [&](int sub) {
    seg_end = min(re, b_end);
    split = b_start < rs || b_end > re;
    int ec;
    frexpf((float)(b_end - b_start) + 1.0f, &ec);                  // count < 2^ec
    const int e = 61 - ev - ec;
    up = ldexp(1.0, e);
    down = ldexp(1.0, -e);
    base = ((uint32_t)B << a.bin_shift) + ((uint32_t)sub << kBinBits);
    lim = min((int64_t)NB, a.n_entries - (int64_t)base);
  };

  if (a.n_sub == 1) {
    // One continuous stream over [rs, re) in chunks of CH records, the next chunk's loads in flight
    // while the current one is added (two record buffers taking turns, so no register copies wait
    // for loads); a segment ends (barrier, flush, barrier) wherever its bin ends.  Record loads are
    // unpredicated (positions past re re-read record re - 1, which is never added) so that the wait
    // for the current chunk leaves the next chunk's loads outstanding.  Each record is read exactly
    // once, so the loads are non-temporal: the stream then does not evict the parameters, moments
    // and table lines of the flushes and of the next step's encoder from the L2s and the memory-side
    // cache.
    auto load = [&](BinRec (&buf)[U], uint32_t cb) {
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const BinRec* r = a.recs + min(cb + k * kReduceThreads + threadIdx.x, re - 1);
        buf[k].idx = __builtin_nontemporal_load(&r->idx);
        buf[k].v0 = __builtin_nontemporal_load(&r->v0);
        buf[k].v1 = __builtin_nontemporal_load(&r->v1);
      }
    };
    auto add_chunk = [&](const BinRec (&cur)[U], uint32_t cb) {
      const uint32_t ce = min(re, cb + CH);
      uint32_t lo = cb;
      for (;;) {
        const uint32_t hi = min(seg_end, ce);
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const uint32_t r = cb + k * kReduceThreads + threadIdx.x;
          if (r >= lo && r < hi) rec_add(tile64, cur[k], base, up);
        }
        if (seg_end > ce) return;                                  // the segment goes on in the next chunk
        __syncthreads();
        tile_flush<FUSED>(a, tile64, base, lim, split, 2 * (size_t)jb + (B == first_bin ? 0 : 1), 0, down);
        __syncthreads();
        if (seg_end >= re) return;                                 // the block's range is done
        lo = seg_end;
        do {                                                       // next bin with records
          ++B;
          b_start = b_end;
          b_end = bstart(B + 1);
        } while (b_end <= b_start);
        begin_segment(0);
        if (lo >= ce) return;
      }
    };
    begin_segment(0);
    BinRec buf0[U], buf1[U];
    load(buf0, rs);
    for (uint32_t cb = rs; cb < re; cb += 2 * CH) {
      load(buf1, cb + CH);
      add_chunk(buf0, cb);
      if (cb + CH >= re) break;
      load(buf0, cb + 2 * CH);
      add_chunk(buf1, cb + CH);
    }
    return;
  }

  // Bins of several tiles: each segment is streamed once per tile.
  uint32_t pos = rs;
  for (;;) {
    for (int sub = 0; sub < a.n_sub; ++sub) {
      begin_segment(sub);
      const BinRec* __restrict__ src = a.recs + pos;
      const int cnt = (int)(seg_end - pos);
      for (int r0 = 0; r0 < cnt; r0 += CH) {
        BinRec rc[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const int r = r0 + k * kReduceThreads + threadIdx.x;
          if (r < cnt) rc[k] = src[r];
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
          if (r0 + k * kReduceThreads + (int)threadIdx.x < cnt) rec_add(tile64, rc[k], base, up);
      }
      __syncthreads();
      tile_flush<FUSED>(a, tile64, base, lim, split, 2 * (size_t)jb + (B == first_bin ? 0 : 1), sub, down);
      __syncthreads();
    }
    pos = seg_end;
    if (pos >= re) break;
    do {
      ++B;
      b_start = b_end;
      b_end = bstart(B + 1);
    } while (b_end <= b_start);
  }
}

// Bins cut by the range boundaries of k_bin_reduce: block j (1 <= j < G') takes the bin holding
// record block_start[j] when that bin starts inside block j - 1's range, adds the int64 slots of the
// blocks j0 = j - 1 .. j1 that hold part of it in order, and adds the result to the FP32 gradient.
// Each such block j is kCombineParts blocks here, part k taking the k-th part of every tile (short
// chains of loads per thread instead of eight entries each), and the grid is a.ray_blocks blocks
// drawing the next training step's rays, then kCombineParts x the reduction's grid G, then
// a.dense_blocks blocks of the dense gradient reduction.
__global__ void __launch_bounds__(1024) k_bin_combine(const BinReduceArgs a) {
  constexpr int NB = 1 << kBinBits, QP = NB / kCombineParts;
  __shared__ float red[1024];
  if ((int)blockIdx.x < a.ray_blocks) {   // the next training step's rays (block-uniform)
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < a.next_rays.n_rays) ray_one(a.next_rays, r);
    return;
  }
  const int bx = (int)blockIdx.x - a.ray_blocks;
  const int GP = (int)gridDim.x - a.ray_blocks - a.dense_blocks, G = GP / kCombineParts;
  if (bx >= GP) {   // block-uniform
    dense_reduce_block(a.dense, bx - GP, red);
    return;
  }
  if (*a.bad_step) return;   // non-finite step: write nothing (block-uniform)
  const int part = bx % kCombineParts, q0 = part * QP;
  if (a.fused) {   // bins without records: Adam with a zero gradient (dense Adam semantics)
    for (int B = bx / kCombineParts; B < a.n_bins; B += G) {
      if (a.bin_start[B] != a.bin_start[B + 1]) continue;
      for (int sub = 0; sub < a.n_sub; ++sub) {
        const uint32_t base = ((uint32_t)B << a.bin_shift) + ((uint32_t)sub << kBinBits);
        const int64_t lim = min((int64_t)NB, a.n_entries - (int64_t)base);
        for (int q = q0 + threadIdx.x; q < min((int64_t)(q0 + QP), lim); q += blockDim.x) {
          float2 pp = reinterpret_cast<float2*>(a.p)[base + q], mm = reinterpret_cast<float2*>(a.m)[base + q],
                 vv = reinterpret_cast<float2*>(a.v)[base + q];
          adam_update(pp.x, mm.x, vv.x, 0.0f, a.adam);
          adam_update(pp.y, mm.y, vv.y, 0.0f, a.adam);
          reinterpret_cast<float2*>(a.p)[base + q] = pp;
          reinterpret_cast<float2*>(a.m)[base + q] = mm;
          reinterpret_cast<float2*>(a.v)[base + q] = vv;
          if (a.th) reinterpret_cast<__half2*>(a.th)[base + q] = __floats2half2_rn(pp.x, pp.y);
        }
      }
    }
  }
  const uint64_t T = a.bin_start[a.n_bins];
  const uint64_t Ge = T < (uint64_t)G ? T : (uint64_t)G;
  const uint64_t jb = bx / kCombineParts;
  if (jb == 0 || jb >= Ge) return;
  const uint32_t rs = a.block_start[jb], rs_prev = a.block_start[jb - 1];
  if (rs >= T) return;
  const int B = a.block_first_bin[jb];
  const uint32_t b_start = a.bin_start[B], b_end = a.bin_start[B + 1];
  if (!(b_start < rs && b_start >= rs_prev)) return;     // not cut here, or cut at an earlier boundary
  const uint32_t j0 = (uint32_t)jb - 1;
  uint32_t j1 = (uint32_t)jb;                            // the last block whose range reaches into the bin
  while (j1 + 1 < Ge && a.block_start[j1 + 1] < b_end) ++j1;
  const float vmax = __uint_as_float(*a.rec_max_bits);
  int ev, ec;
  frexpf(vmax, &ev);
  frexpf((float)(b_end - b_start) + 1.0f, &ec);
  const double down = ldexp(1.0, -(61 - ev - ec));
  const int n_sub = a.n_sub;
  for (int sub = 0; sub < n_sub; ++sub) {
    const uint32_t base = ((uint32_t)B << a.bin_shift) + ((uint32_t)sub << kBinBits);
    const int64_t lim = min((int64_t)NB, a.n_entries - (int64_t)base);
    float2* g2 = reinterpret_cast<float2*>(a.grad_table) + base;
    for (int q = q0 + threadIdx.x; q < min((int64_t)(q0 + QP), lim); q += blockDim.x) {
      long long s0 = 0, s1 = 0;
      for (uint32_t jj = j0; jj <= j1; ++jj) {
        if (a.block_start[jj] == a.block_start[jj + 1]) continue;   // an empty range wrote no slot
        const size_t sl = 2 * (size_t)jj + (a.block_first_bin[jj] == B ? 0 : 1);
        const unsigned long long* S = a.split_acc + (sl * n_sub + sub) * (2 * NB);
        s0 += (long long)S[2 * q];
        s1 += (long long)S[2 * q + 1];
      }
      const float d0 = (float)((double)s0 * down), d1 = (float)((double)s1 * down);
      if (a.fused) {
        float2 pp = reinterpret_cast<float2*>(a.p)[base + q], mm = reinterpret_cast<float2*>(a.m)[base + q],
               vv = reinterpret_cast<float2*>(a.v)[base + q];
        adam_update(pp.x, mm.x, vv.x, d0, a.adam);
        adam_update(pp.y, mm.y, vv.y, d1, a.adam);
        reinterpret_cast<float2*>(a.p)[base + q] = pp;
        reinterpret_cast<float2*>(a.m)[base + q] = mm;
        reinterpret_cast<float2*>(a.v)[base + q] = vv;
        if (a.th) reinterpret_cast<__half2*>(a.th)[base + q] = __floats2half2_rn(pp.x, pp.y);
      } else {
        float2 o = g2[q];
        o.x += d0;
        o.y += d1;
        g2[q] = o;
      }
    }
  }
}

// Per-block FP64 sums of squared errors and maxima of gt (for PSNR): partials[2b] = sum,
// partials[2b + 1] = max.
__global__ void __launch_bounds__(256) k_sqerr(const float* __restrict__ gt, const float* __restrict__ pred,
                                               int64_t n, double* __restrict__ partials) {
  __shared__ double ss[256], sm[256];
  double s = 0.0, mx = -1e300;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    const double d = (double)pred[q] - (double)gt[q];
    s += d * d;
    mx = fmax(mx, (double)gt[q]);
  }
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      ss[threadIdx.x] += ss[threadIdx.x + o];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = ss[0];
    partials[2 * blockIdx.x + 1] = sm[0];
  }
}

// 3-D SSIM (Wang et al. 2004 extended to volumes): local statistics under a separable Gaussian
// window (sigma 1.5, radius 5, weights normalised to sum 1), C1 = (0.01 L)^2, C2 = (0.03 L)^2, over
// the voxels whose whole window lies inside the volume; FP64 throughout.  Grid-stride over those
// voxels; partials[b] = the block's sum of SSIM terms (fixed order: per thread, then a tree).
__global__ void __launch_bounds__(256) k_ssim(const float* __restrict__ gt, const float* __restrict__ pred,
                                              int nx, int ny, int nz, double c1, double c2,
                                              double* __restrict__ partials) {
  constexpr int R = 5;
  __shared__ double w[2 * R + 1];
  __shared__ double red[256];
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = -R; i <= R; ++i) s += exp(-(double)(i * i) / (2.0 * 1.5 * 1.5));
    for (int i = -R; i <= R; ++i) w[i + R] = exp(-(double)(i * i) / (2.0 * 1.5 * 1.5)) / s;
  }
  __syncthreads();
  const int vx = nx - 2 * R, vy = ny - 2 * R, vz = nz - 2 * R;
  const int64_t nv = (int64_t)vx * vy * vz;
  double term = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nv; q += (int64_t)gridDim.x * blockDim.x) {
    const int x = (int)(q % vx) + R;
    const int y = (int)((q / vx) % vy) + R;
    const int z = (int)(q / ((int64_t)vx * vy)) + R;
    double sa = 0.0, sb = 0.0, saa = 0.0, sbb = 0.0, sab = 0.0;
    for (int dz = -R; dz <= R; ++dz) {
      for (int dy = -R; dy <= R; ++dy) {
        const double wzy = w[dz + R] * w[dy + R];
        const int64_t row = ((int64_t)(z + dz) * ny + (y + dy)) * nx;
        for (int dx = -R; dx <= R; ++dx) {
          const double ww = wzy * w[dx + R];
          const double a = gt[row + x + dx], b = pred[row + x + dx];
          sa += ww * a;
          sb += ww * b;
          saa += ww * a * a;
          sbb += ww * b * b;
          sab += ww * a * b;
        }
      }
    }
    const double va = saa - sa * sa, vb = sbb - sb * sb, cab = sab - sa * sb;
    term += ((2.0 * sa * sb + c1) * (2.0 * cab + c2)) / ((sa * sa + sb * sb + c1) * (va + vb + c2));
  }
  red[threadIdx.x] = term;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------------------------
// Channel spectra (Sec. 2.3: noisy hash-feature channels are found with an FFT).  For one level of
// resolution N the probe is the G^3 grid of its own vertices v0 + i (i < G = min(Gmax, N)) around the
// box centre; each of the level's channels is sampled there, transformed with a 3-D DFT (FP64), and
// its power split into the high band (max_d |k_d| > G/4, signed frequencies) and the rest (DC
// excluded).
// ---------------------------------------------------------------------------------------------
__global__ void k_probe_points(int N, int v0, int G, float* __restrict__ xn) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)G * G * G) return;
  const int ix = (int)(q % G), iy = (int)((q / G) % G), iz = (int)(q / ((int64_t)G * G));
  xn[3 * q] = (float)(v0 + ix) / (float)N;
  xn[3 * q + 1] = (float)(v0 + iy) / (float)N;
  xn[3 * q + 2] = (float)(v0 + iz) / (float)N;
}

// One DFT pass along axis `axis` (0 = x, fastest) of a G^3 complex field [z][y][x]; the first pass
// reads the real channel c of the encodings enc [G^3][C] instead (in == NULL).
__global__ void k_dft_axis(const double2* __restrict__ in, const float* __restrict__ enc, int C, int c, int G,
                           int axis, double2* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)G * G * G) return;
  const int ix = (int)(q % G), iy = (int)((q / G) % G), iz = (int)(q / ((int64_t)G * G));
  const int k = axis == 0 ? ix : (axis == 1 ? iy : iz);
  const int64_t stride = axis == 0 ? 1 : (axis == 1 ? G : (int64_t)G * G);
  const int64_t base = q - (int64_t)k * stride;
  double re = 0.0, im = 0.0;
  for (int n = 0; n < G; ++n) {
    const int64_t src = base + (int64_t)n * stride;
    const double2 v = in ? in[src] : make_double2((double)enc[src * C + c], 0.0);
    const int j = (int)(((int64_t)k * n) % G);
    double sn, cs;
    sincospi(2.0 * (double)j / (double)G, &sn, &cs);
    re += v.x * cs + v.y * sn;          // v * exp(-2 pi i k n / G)
    im += v.y * cs - v.x * sn;
  }
  out[q] = make_double2(re, im);
}

// Per-block FP64 sums of the power in the high band (partials[2b]) and of all non-DC power
// (partials[2b + 1]).
__global__ void __launch_bounds__(256) k_band_power(const double2* __restrict__ X, int G,
                                                    double* __restrict__ partials) {
  __shared__ double sh[256], st[256];
  double hi = 0.0, tot = 0.0;
  const int64_t n = (int64_t)G * G * G;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    if (q == 0) continue;
    const int k[3] = {(int)(q % G), (int)((q / G) % G), (int)(q / ((int64_t)G * G))};
    int kmax = 0;
    for (int d = 0; d < 3; ++d) {
      const int s = k[d] <= G / 2 ? k[d] : G - k[d];
      kmax = s > kmax ? s : kmax;
    }
    const double p = X[q].x * X[q].x + X[q].y * X[q].y;
    tot += p;
    if (4 * kmax > G) hi += p;
  }
  sh[threadIdx.x] = hi;
  st[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sh[threadIdx.x] += sh[threadIdx.x + o];
      st[threadIdx.x] += st[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sh[0];
    partials[2 * blockIdx.x + 1] = st[0];
  }
}

hipError_t launch_probe_points(int N, int v0, int G, float* xn, hipStream_t s) {
  const int64_t n = (int64_t)G * G * G;
  k_probe_points<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(N, v0, G, xn);
  return hipGetLastError();
}

hipError_t launch_channel_power(const float* enc, int C, int c, int G, double2* b0, double2* b1, double* partials,
                                int n_blocks, hipStream_t s) {
  const int64_t n = (int64_t)G * G * G;
  const unsigned g = (unsigned)((n + 255) / 256);
  k_dft_axis<<<g, 256, 0, s>>>(nullptr, enc, C, c, G, 0, b0);
  k_dft_axis<<<g, 256, 0, s>>>(b0, nullptr, C, c, G, 1, b1);
  k_dft_axis<<<g, 256, 0, s>>>(b1, nullptr, C, c, G, 2, b0);
  k_band_power<<<n_blocks, 256, 0, s>>>(b0, G, partials);
  return hipGetLastError();
}

// Raw encoding of n points (all levels, natural channel order) and optional corner entries.
__global__ void k_encode(const LevelTab lt, const void* __restrict__ table, int half_table,
                         const float* __restrict__ xn, int64_t n, float* __restrict__ enc,
                         uint32_t* __restrict__ idx_out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * lt.L) return;
  const int64_t p = q / lt.L;
  const int l = (int)(q - p * lt.L);
  const float x[3] = {xn[3 * p], xn[3 * p + 1], xn[3 * p + 2]};
  uint32_t idx[8];
  float w[8];
  level_corners(lt.res[l], lt.off[l], lt.stride[l], lt.mask, x, idx, w);
  float s0 = 0.0f, s1 = 0.0f;
  for (int c = 0; c < 8; ++c) {
    const float2 v = half_table ? __half22float2(reinterpret_cast<const __half2*>(table)[idx[c]])
                                : reinterpret_cast<const float2*>(table)[idx[c]];
    s0 += w[c] * v.x;
    s1 += w[c] * v.y;
  }
  enc[p * 2 * lt.L + 2 * l] = s0;
  enc[p * 2 * lt.L + 2 * l + 1] = s1;
  if (idx_out)
    for (int c = 0; c < 8; ++c) idx_out[(p * lt.L + l) * 8 + c] = idx[c];
}

// ---------------------------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------------------------
template <int L, int W, int D, int P>
static KernelSet make_set() {
  constexpr int C = 2 * L;
  using Ly = Lay<C, W, D, P>;
  KernelSet ks;
  ks.fwd = reinterpret_cast<const void*>(&k_fwd<L, W, D, P, false>);
  ks.fwd_pre = reinterpret_cast<const void*>(&k_fwd<L, W, D, P, true>);
  ks.bwd = reinterpret_cast<const void*>(&k_bwd<L, W, D, P>);
  ks.enc = reinterpret_cast<const void*>(&k_enc<L, P>);
  ks.fwd_lds = Ly::s_n * sizeof(float);
  const int nd_pad = (Ly::g_n + 3) & ~3;
  ks.bwd_lds = (Ly::s_n + bwd_tiles_lds<W>(nd_pad)) * sizeof(float);
  ks.n_dense = Ly::g_n;
  ks.nd_pad = nd_pad;
  ks.valid = true;
  return ks;
}

KernelSet kernel_set(int L, int W, int D, int precision) {
#define NIC_CASE(l, w, d)                                      \
  if (L == l && W == w && D == d)                              \
    return precision ? make_set<l, w, d, 1>() : make_set<l, w, d, 0>();
  NIC_CASE(8, 32, 1) NIC_CASE(8, 32, 2) NIC_CASE(8, 32, 3) NIC_CASE(8, 32, 4)
  NIC_CASE(16, 32, 1) NIC_CASE(16, 32, 2) NIC_CASE(16, 32, 3) NIC_CASE(16, 32, 4)
  NIC_CASE(8, 64, 4) NIC_CASE(16, 64, 4)
#undef NIC_CASE
  return KernelSet{};
}

hipError_t launch_fwd(const KernelSet& ks, const FwdArgs& a, int max_grid, size_t extra_lds, hipStream_t s) {
  int64_t blocks = (a.n_points + kPtsPerBlock - 1) / kPtsPerBlock;
  if (blocks == 0) return hipSuccess;
  if (max_grid > 0 && blocks > max_grid) blocks = max_grid;
  if (a.enc_pre && (a.mode != kModeRays || a.bin_counts || a.enc_out)) return hipErrorInvalidValue;
  void* args[] = {const_cast<FwdArgs*>(&a)};
  return hipLaunchKernel(a.enc_pre ? ks.fwd_pre : ks.fwd, dim3((unsigned)blocks), dim3(kBlock), args,
                         ks.fwd_lds + extra_lds, s);
}

hipError_t launch_bwd(const KernelSet& ks, const FwdArgs& a, const BwdArgs& b, int grid, size_t extra_lds,
                      hipStream_t s) {
  void* args[] = {const_cast<FwdArgs*>(&a), const_cast<BwdArgs*>(&b)};
  return hipLaunchKernel(ks.bwd, dim3((unsigned)grid), dim3(kBlock), args, ks.bwd_lds + extra_lds, s);
}

hipError_t launch_enc(const KernelSet& ks, const FwdArgs& a, size_t lds, hipStream_t s) {
  if (a.n_points == 0) return hipSuccess;
  if (a.enc_grid < 1 || !a.enc_out || !a.bin_counts || !a.edge_counts || a.mode != kModeRays)
    return hipErrorInvalidValue;
  const int64_t blocks = 8ll * ((a.lt.L + 7) / 8) * a.enc_grid;
  void* args[] = {const_cast<FwdArgs*>(&a)};
  return hipLaunchKernel(ks.enc, dim3((unsigned)blocks), dim3(kEncThreads), args, lds, s);
}

hipError_t launch_rays(const RaysArgs& a, hipStream_t s) {
  if (a.n_rays == 0) return hipSuccess;
  k_rays<<<(a.n_rays + 127) / 128, 128, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_raysum(const float* ws, int wpr, int n_rays, float* out, hipStream_t s) {
  if (n_rays == 0) return hipSuccess;
  k_raysum<<<(n_rays + 255) / 256, 256, 0, s>>>(ws, wpr, n_rays, out);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float* x, int64_t n, uint32_t* count, int n_cu, hipStream_t s) {
  k_fill<<<1, 64, 0, s>>>(reinterpret_cast<float*>(count), 1, 0.0f);   // bits of 0.0f are 0
  if (n == 0) return hipGetLastError();
  int64_t blocks = (n + 255) / 256;
  if (blocks > (int64_t)n_cu * 8) blocks = (int64_t)n_cu * 8;
  k_count_nonfinite<<<(unsigned)blocks, 256, 0, s>>>(x, n, count);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float ibc1, float ibc2, __half* th, int64_t n_table, const uint32_t* bad_step,
                       int n_cu, hipStream_t s) {
  const int64_t n4 = n / 4;
  int64_t blocks = (n4 + 255) / 256;
  const int64_t cap = (int64_t)n_cu * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  k_adam<<<(unsigned)blocks, 256, 0, s>>>(reinterpret_cast<float4*>(p), reinterpret_cast<float4*>(g),
                                          reinterpret_cast<float4*>(m), reinterpret_cast<float4*>(v), n4, lr, b1,
                                          b2, eps, ibc1, ibc2, th, n_table, bad_step);
  return hipGetLastError();
}

hipError_t launch_fill(float* x, int64_t n, float val, int n_cu, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > (int64_t)n_cu * 16) blocks = (int64_t)n_cu * 16;
  k_fill<<<(unsigned)blocks, 256, 0, s>>>(x, n, val);
  return hipGetLastError();
}

hipError_t launch_to_half(const float* src, __half* dst, int64_t n, int n_cu, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > (int64_t)n_cu * 16) blocks = (int64_t)n_cu * 16;
  k_to_half<<<(unsigned)blocks, 256, 0, s>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_init(float* params, int64_t n_table, int64_t dense_off, const InitArgs& ia, int n_cu,
                       hipStream_t s) {
  int64_t blocks = (n_table + 255) / 256;
  if (blocks > (int64_t)n_cu * 16) blocks = (int64_t)n_cu * 16;
  if (blocks < 1) blocks = 1;
  k_init<<<(unsigned)blocks, 256, 0, s>>>(params, n_table, dense_off, ia);
  return hipGetLastError();
}

hipError_t launch_bin_scan(const uint32_t* counts, int n_bins, int grid, uint32_t* rel, uint32_t* totals,
                           uint32_t* bin_start, uint32_t* block_start, int32_t* block_first_bin, int reduce_grid,
                           uint32_t* rec_max_bits, const uint32_t* edge, const int32_t* edge_beg,
                           const int32_t* edge_src, bool rows_done, hipStream_t s) {
  if (!rows_done) k_bin_rowscan<<<n_bins, 256, 0, s>>>(counts, grid, rel, totals, edge, edge_beg, edge_src);
  k_bin_plan<<<1, 1024, 0, s>>>(totals, n_bins, reduce_grid, bin_start, block_start, block_first_bin, rec_max_bits);
  return hipGetLastError();
}

size_t bin_reduce_lds() { return (size_t)2 * (1 << kBinBits) * sizeof(unsigned long long); }

hipError_t launch_bin_reduce(const BinReduceArgs& a, int grid, hipStream_t s) {
  if (a.bin_shift < kBinBits || a.bin_shift > 31 || a.n_sub != (1 << (a.bin_shift - kBinBits)))
    return hipErrorInvalidValue;
  if (a.dense_blocks != (a.dense.nd + 63) / 64) return hipErrorInvalidValue;
  if (a.ray_blocks != (a.next_rays.n_rays + 1023) / 1024) return hipErrorInvalidValue;
  if (a.fused) k_bin_reduce<true><<<grid, kReduceThreads, bin_reduce_lds(), s>>>(a);
  else k_bin_reduce<false><<<grid, kReduceThreads, bin_reduce_lds(), s>>>(a);
  k_bin_combine<<<a.ray_blocks + kCombineParts * grid + a.dense_blocks, 1024, 0, s>>>(a);
  return hipGetLastError();
}

const void* bin_reduce_kernel(bool fused) {
  return fused ? reinterpret_cast<const void*>(&k_bin_reduce<true>) : reinterpret_cast<const void*>(&k_bin_reduce<false>);
}

hipError_t launch_ssim(const float* gt, const float* pred, int nx, int ny, int nz, double c1, double c2,
                       double* partials, int n_blocks, hipStream_t s) {
  k_ssim<<<n_blocks, 256, 0, s>>>(gt, pred, nx, ny, nz, c1, c2, partials);
  return hipGetLastError();
}

hipError_t launch_sqerr(const float* gt, const float* pred, int64_t n, double* partials, int n_blocks,
                        hipStream_t s) {
  k_sqerr<<<n_blocks, 256, 0, s>>>(gt, pred, n, partials);
  return hipGetLastError();
}

hipError_t launch_encode(const LevelTab& lt, const void* table, int half_table, const float* xn, int64_t n,
                         float* enc, uint32_t* idx, hipStream_t s) {
  const int64_t tot = n * lt.L;
  if (tot == 0) return hipSuccess;
  k_encode<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(lt, table, half_table, xn, n, enc, idx);
  return hipGetLastError();
}

}  // namespace nic
