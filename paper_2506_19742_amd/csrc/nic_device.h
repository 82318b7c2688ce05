// Device building blocks of libnic for gfx950: counter-based draws, cone-beam ray setup and
// sampling, multiresolution hash encoding, and the 32x32 MFMA tiles of the MLP.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace nic {

constexpr int kMaxLevels = 16;
constexpr int kWave = 64;
constexpr int kPtsPerWave = 32;      // two lanes per point: lane half h = lane >> 5
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kPtsPerBlock = kPtsPerWave * kWavesPerBlock;
constexpr int kEncThreads = 256;     // level-major encoder: one lane per point, two chunks at once
static_assert(kEncThreads % kPtsPerBlock == 0, "the encoder takes whole chunks");
constexpr int kTile = 33;            // padded row length of the per-wave LDS transpose tiles
constexpr int kBinBits = 13;         // reduction tile: 2^13 entries (128 KB of int64 x 2 in LDS)
// A table-gradient bin spans 2^bin_shift entries, bin_shift >= kBinBits, chosen per model so that
// the per-bin histogram fits in LDS beside the kernels' own tiles; a bin of more than one tile is
// reduced tile by tile.
constexpr int kLdsBytes = 160 * 1024;
constexpr int kReduceThreads = 1024;  // threads of a bin-reduction block
constexpr int kBinTilePer = (1 << kBinBits) / kReduceThreads;  // tile entries per thread
constexpr unsigned kFlushCost = 32768;  // a tile flush costs about as much time as streaming this many records
constexpr int kCombineParts = 4;        // k_bin_combine blocks per cut bin (each takes a quarter of every tile)

// One corner contribution to the table gradient: entry and the two feature gradients.
struct BinRec {
  uint32_t idx;
  float v0, v1;
};

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Philox4x32-10 stream ids (fourth counter word).
enum : uint32_t { kJitter = 1, kRays = 2, kViews = 3, kTable = 4, kMlp = 5, kPoints = 6 };

// ---------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64 multiplies with
// the key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------------------------
__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}

__host__ __device__ inline uint32_t philox_w0(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3) {
  uint32_t c[4] = {c0, c1, c2, c3};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  return c[0];
}

// 24-bit uniform in [0, 1).
__host__ __device__ inline float u24f(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

__device__ inline float jitter(uint64_t seed, uint32_t step, uint32_t slot, uint32_t i) {
  return u24f(philox_w0(seed, i, slot, step, kJitter));
}

// Four-round balanced Feistel bijection on [0, 2^(2h)) keyed by (seed, step); round function =
// first Philox word of (right half, round, step, stream) masked to h bits.
__device__ inline uint32_t feistel(uint64_t seed, uint32_t step, int h, uint32_t x) {
  const uint32_t mask = (1u << h) - 1u;
  uint32_t L = (x >> h) & mask, R = x & mask;
  for (uint32_t rnd = 0; rnd < 4; ++rnd) {
    const uint32_t f = philox_w0(seed, R, rnd, step, kRays) & mask;
    const uint32_t nR = L ^ f;
    L = R;
    R = nR;
  }
  return (L << h) | R;
}

// Pixel of ray slot j: the bijection restricted to [0, n_pix) by cycle walking (distinct slots give
// distinct pixels).  The walk ends because j < n_pix lies on the same cycle.
__device__ inline int32_t draw_pixel(uint64_t seed, uint32_t step, int h, uint32_t n_pix, uint32_t j) {
  uint32_t y = feistel(seed, step, h, j);
  while (y >= n_pix) y = feistel(seed, step, h, y);
  return (int32_t)y;
}

// ---------------------------------------------------------------------------------------------
// Cone-beam ray (circular orbit about z) and stratified samples.  The sequence of FP64 operations
// is fixed and contraction is off, so every normalised FP32 sample position is reproducible.
// ---------------------------------------------------------------------------------------------
struct Geo {
  double dso, back;            // back = dsd - dso
  double du, dv, off_u, off_v;
  double vol[3], inv_vol[3];
  int32_t nu, nv;
};

struct RayRec {                // 80 bytes, one per ray slot
  double s[3];
  double d[3];                 // pixel - source
  double t0, dt;               // segment start and bin length (in units of |d|)
  float delta;                 // bin length in mm
  float a_gt;                  // measured line integral of the pixel
  int32_t hit;
  int32_t pix;
};

__device__ inline void ray_setup(const Geo& g, double ca, double sa, int32_t pix, int N, RayRec& r) {
#pragma clang fp contract(off)
  const int32_t row = pix / g.nu, col = pix % g.nu;
  const double s0 = g.dso * ca, s1 = g.dso * sa, s2 = 0.0;
  const double dc0 = -(g.back * ca), dc1 = -(g.back * sa);
  const double u = (((double)col + 0.5) - 0.5 * (double)g.nu) * g.du + g.off_u;
  const double v = (((double)row + 0.5) - 0.5 * (double)g.nv) * g.dv + g.off_v;
  const double P0 = dc0 + u * (-sa);
  const double P1 = dc1 + u * ca;
  const double P2 = v;
  const double s[3] = {s0, s1, s2};
  const double d[3] = {P0 - s0, P1 - s1, P2 - s2};
  double lo = 0.0, hi = 1.0;
  int hit = 1;
  for (int k = 0; k < 3; ++k) {
    const double bl = -0.5 * g.vol[k], bh = 0.5 * g.vol[k];
    if (d[k] != 0.0) {
      const double ta = (bl - s[k]) / d[k];
      const double tb = (bh - s[k]) / d[k];
      const double tn = ta < tb ? ta : tb;
      const double tf = ta < tb ? tb : ta;
      if (tn > lo) lo = tn;
      if (tf < hi) hi = tf;
    } else if (s[k] < bl || s[k] > bh) {
      hit = 0;
    }
  }
  if (!(hi > lo)) hit = 0;
  const double len = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
  const double dt = (hi - lo) / (double)N;
  for (int k = 0; k < 3; ++k) { r.s[k] = s[k]; r.d[k] = d[k]; }
  r.t0 = lo;
  r.dt = dt;
  r.delta = hit ? (float)(dt * len) : 0.0f;
  r.hit = hit;
  r.pix = pix;
}

// Normalised FP32 position of sample i with jitter u of a hit ray.
__device__ inline void sample_pos(const Geo& g, const RayRec& r, int i, float u, float x[3]) {
#pragma clang fp contract(off)
  const double t = r.t0 + ((double)i + (double)u) * r.dt;
  for (int k = 0; k < 3; ++k) {
    const double xw = r.s[k] + t * r.d[k];
    double xr = (xw + 0.5 * g.vol[k]) * g.inv_vol[k];
    xr = xr < 0.0 ? 0.0 : xr;
    xr = xr > 1.0 ? 1.0 : xr;
    x[k] = (float)xr;
  }
}

// Point p of step `step` for the voxel loss: three 24-bit uniforms from one Philox block.
__device__ inline void voxel_point(uint64_t seed, uint32_t step, uint32_t p, float x[3]) {
  uint32_t c[4] = {p, step, 0u, kPoints};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  x[0] = u24f(c[0]);
  x[1] = u24f(c[1]);
  x[2] = u24f(c[2]);
}

// Trilinear sample of vol[z][y][x] (n^3 voxels, centres at (i + 1/2)/n) at a normalised point:
// continuous index u = x n - 1/2 clamped to [0, n - 1], base cell floor(u) clamped to n - 2.
__device__ inline float trilinear(const float* __restrict__ vol, int n, const float x[3]) {
  int b[3];
  float f[3];
  for (int k = 0; k < 3; ++k) {
    float u = x[k] * (float)n - 0.5f;
    u = u < 0.0f ? 0.0f : u;
    u = u > (float)(n - 1) ? (float)(n - 1) : u;
    int i = (int)floorf(u);
    i = i > n - 2 ? n - 2 : i;
    i = i < 0 ? 0 : i;
    b[k] = i;
    f[k] = u - (float)i;
  }
  float s = 0.0f;
  for (int c = 0; c < 8; ++c) {
    const int c0 = c & 1, c1 = (c >> 1) & 1, c2 = (c >> 2) & 1;
    const float w = (c0 ? f[0] : 1.0f - f[0]) * (c1 ? f[1] : 1.0f - f[1]) * (c2 ? f[2] : 1.0f - f[2]);
    s += w * vol[((size_t)(b[2] + c2) * n + (b[1] + c1)) * n + (b[0] + c0)];
  }
  return s;
}

// Normalised FP32 coordinate of voxel centre i of n along one axis.
__device__ inline float voxel_coord(int i, int n) {
#pragma clang fp contract(off)
  return (float)(((double)i + 0.5) / (double)n);
}

// ---------------------------------------------------------------------------------------------
// Multiresolution hash grid
// ---------------------------------------------------------------------------------------------
struct LevelTab {
  int32_t res[kMaxLevels];
  uint32_t off[kMaxLevels];
  uint32_t stride[kMaxLevels];   // N_l + 1 for a dense level, 0 for a hashed level
  uint32_t mask;                 // T - 1
  int32_t L;
  int32_t bin_shift;             // log2 of the entries per table-gradient bin
  uint32_t on;                   // bit l: level l is used (a level whose two channels are masked is not)
};

// Cell g = min(floor(fl32(x * N)), N - 1) and fraction f = x*N - g (exact) along one axis.
__device__ __forceinline__ void cell_of(float x, int32_t N, uint32_t& g, float& f) {
  const float pos = __fmul_rn(x, (float)N);
  int32_t gi = (int32_t)floorf(pos);
  gi = gi > N - 1 ? N - 1 : gi;
  gi = gi < 0 ? 0 : gi;
  g = (uint32_t)gi;
  f = __fsub_rn(pos, (float)gi);
}

// Global entries and trilinear weights of the 8 corners (c = c0 + 2 c1 + 4 c2) of one level.
// Dense: off + v0 + s (v1 + s v2), s = N + 1.  Hashed: off + ((v0 * 1) ^ (v1 * 2654435761) ^
// (v2 * 805459861)) & (T - 1) in uint32 arithmetic (Instant-NGP's spatial hash).
__device__ __forceinline__ void level_corners(int32_t N, uint32_t off, uint32_t stride, uint32_t mask,
                                              const float x[3], uint32_t idx[8], float w[8], uint32_t& g0,
                                              uint32_t& g1, uint32_t& g2) {
  float f0, f1, f2;
  cell_of(x[0], N, g0, f0);
  cell_of(x[1], N, g1, f1);
  cell_of(x[2], N, g2, f2);
  const float wx[2] = {1.0f - f0, f0}, wy[2] = {1.0f - f1, f1}, wz[2] = {1.0f - f2, f2};
  if (stride) {
    const uint32_t a0 = off + g0, b0 = stride * g1, c0 = stride * stride * g2;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      idx[c] = a0 + (c & 1) + b0 + ((c >> 1) & 1) * stride + c0 + ((c >> 2) & 1) * stride * stride;
  } else {
    const uint32_t hx[2] = {g0, g0 + 1u};
    const uint32_t hy[2] = {g1 * 2654435761u, (g1 + 1u) * 2654435761u};
    const uint32_t hz[2] = {g2 * 805459861u, (g2 + 1u) * 805459861u};
#pragma unroll
    for (int c = 0; c < 8; ++c)
      idx[c] = off + ((hx[c & 1] ^ hy[(c >> 1) & 1] ^ hz[(c >> 2) & 1]) & mask);
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) w[c] = wx[c & 1] * wy[(c >> 1) & 1] * wz[(c >> 2) & 1];
}

__device__ __forceinline__ void level_corners(int32_t N, uint32_t off, uint32_t stride, uint32_t mask,
                                              const float x[3], uint32_t idx[8], float w[8]) {
  uint32_t g0, g1, g2;
  level_corners(N, off, stride, mask, x, idx, w, g0, g1, g2);
}

// Runs along a ray: the 32 lanes of a half hold 32 consecutive samples of one ray, so samples that
// share a cell of a coarse level form contiguous runs.  cont: this lane's cell equals the previous
// lane's; tail: the next lane does not continue the run (the run's last lane).
__device__ __forceinline__ void run_flags(uint32_t g0, uint32_t g1, uint32_t g2, int ln, bool& cont, bool& tail) {
  const uint32_t p0 = __shfl_up(g0, 1, 32), p1 = __shfl_up(g1, 1, 32), p2 = __shfl_up(g2, 1, 32);
  cont = ln > 0 && p0 == g0 && p1 == g1 && p2 == g2;
  const int nc = __shfl_down((int)cont, 1, 32);
  tail = !(ln < 31 && nc);
}

// ---------------------------------------------------------------------------------------------
// MFMA 32x32 tiles.  With two lanes per point (point n = lane & 31, half h = lane >> 5), the
// v_mfma_f32_32x32x2f32 output register r of lane half h holds row 8(r/4) + 4h + (r%4) of the
// 32x32 tile.  Every per-point vector (encoding, activations, their gradients) is kept in that
// layout: register R of half h holds channel chan(R, h), so a layer's output feeds the next layer's
// B operand register by register with no cross-lane traffic.
// ---------------------------------------------------------------------------------------------
__host__ __device__ constexpr int chan(int R, int h) {
  return 32 * (R >> 4) + 8 * ((R & 15) >> 2) + 4 * h + (R & 3);
}

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x16 mfma32_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float xor32(float v) { return __shfl_xor(v, 32, 64); }

// Adam (Kingma and Ba, Algorithm 1) on one parameter; ibc1, ibc2 = 1 / (1 - beta^t).  No
// multiply-add contraction: every kernel that runs the update (whichever one a parameter's bin is
// assigned to) rounds it the same way, so a step does not depend on how the work is partitioned.
struct AdamArgs {
  float lr, b1, b2, eps, ibc1, ibc2;
};
__device__ __forceinline__ void adam_update(float& p, float& m, float& v, float g, const AdamArgs& A) {
#pragma clang fp contract(off)
  m = A.b1 * m + (1.0f - A.b1) * g;
  v = A.b2 * v + (1.0f - A.b2) * g * g;
  const float mh = m * A.ibc1, vh = v * A.ibc2;
  p -= A.lr * mh / (sqrtf(vh) + A.eps);
}

// DPP lane moves within rows of 16 lanes (gfx9 encodings): row_shr:n brings lane l - n of the same row
// (0 where that lane is outside the row), row_bcast:15 brings lane 15 of the previous row into rows 1
// and 3 (rows 0 and 2 receive 0).
constexpr int kDppRowShr = 0x110, kDppRowBcast15 = 0x142;
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}

// Sum over the 32 lanes of one half (result in every lane of that half).
__device__ __forceinline__ float half_sum(float v) {
#pragma unroll
  for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The value of v, which the compiler may not assume is the same as at any earlier point: a value
// derived from it is computed where it is used instead of being hoisted out of a loop (and, under
// register pressure, spilled).  Emits no instruction.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Orders this wave's LDS writes before its later LDS reads (and reads before later writes).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace nic
