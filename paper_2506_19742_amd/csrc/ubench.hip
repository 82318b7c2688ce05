// Ceilings of the memory access patterns of the training step on one MI355X (gfx950), each timed
// with HIP events over repeated launches after a warm-up launch:
//   stream_copy / stream_read / stream_write
//                 float4 grid-stride streams over 1 GiB (no index arithmetic beyond the stride),
//                 each at several grid sizes; the best is the stream ceiling
//   copy_l2       float4 copy within a 2 MiB buffer, repeated inside the kernel (L2-resident)
//   encode_*      the encoder's memory work alone: the 16-level hash grid of the 256^3 workload
//                 (T = 2^19, resolutions 16 .. 2048) at the stratified samples of 2048 cone-beam rays
//                 of one view x 192 samples, gathered level-major with the training step's placement
//                 (one lane per point, each XCD on one level at a time) and the encoding stored,
//                 FP32 x 2 or FP16 x 2 entries; encode_lanes_* the same gathers in the layout of a
//                 forward kernel that gathers every level itself (two lanes per point, lane half h
//                 taking half of the levels, all levels on every XCD), for comparison
//   gather_*      random 8-corner cells (four x-adjacent entry pairs, as at a hash-grid level) of
//                 8-B (FP32 x 2) or 4-B (FP16 x 2) entries in tables of 0.94, 48.8 and 169 MB
//   atomic_*      two global f32 atomic adds per corner, spread over a 48.8 MB table or contended
//                 into 4913 entries (the coarsest level)
//   records       streaming read of 33 M 12-byte records (entry, value, value) as the bin reduction
//                 reads them
//   lds_*         random LDS atomic adds (f32, u32, u64) within a 64 KB block-local array
// Every index is reduced into its buffer before use.  Prints one line per measurement; the lines
// starting with "ceiling" are machine-readable (name, value, unit).  With --quick only the stream
// and encode ceilings are measured.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "nic_device.h"

#define UB_CHECK(x)                                                              \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                              \
    }                                                                            \
  } while (0)

namespace {

using namespace nic;

__device__ __forceinline__ unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__global__ void k_stream_copy(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

__global__ void k_stream_read(const float4* __restrict__ a, size_t n, float* __restrict__ out) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  float s = 0.0f;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const float4 v = a[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  if (s == 12345.0f) out[0] = s;   // keeps the loads; never true for the zero-filled buffer
}

__global__ void k_stream_write(float4* __restrict__ b, size_t n, float val) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const float4 v = make_float4(val, val, val, val);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) b[i] = v;
}

// L2-resident copy: reps passes over the same n float4 of a small buffer.
__global__ void k_copy_l2(const float4* __restrict__ a, float4* __restrict__ b, size_t n, int reps) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (int r = 0; r < reps; ++r)
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// Rays of one view through the 256-mm box (DSO 1000 mm, DSD 1500 mm, 256 x 256 detector of 1.5 mm
// pixels), distinct-enough pixels from a hash of the slot.
__global__ void k_ub_rays(Geo g, double ca, double sa, int n_rays, int n_pix, int N, RayRec* __restrict__ rays) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rays) return;
  RayRec rr;
  ray_setup(g, ca, sa, (int32_t)(mix32((unsigned)r * 2654435761u + 7u) % (unsigned)n_pix), N, rr);
  rays[r] = rr;
}

// The encoder's gathers and encoding store alone, placed as in the training step: block b runs on
// XCD x = b mod 8 and takes level 8 * phase + (x, or 7 - x in odd phases) (phase = (b / 8) / G) for
// the points of group w = (b / 8) mod G (chunks w, w + G, ... of kPtsPerBlock points, two at a
// time), one lane per point.
template <bool HALF>
__global__ void __launch_bounds__(kEncThreads) k_encode_lvl(const LevelTab T, const void* __restrict__ table,
                                                            const RayRec* __restrict__ rays, Geo g, int N,
                                                            int64_t n_points, int G, float2* __restrict__ out) {
  const int s = (int)(blockIdx.x >> 3), ph = s / G, w = s - ph * G;
  const int x = (int)(blockIdx.x & 7u);
  const int l = 8 * ph + ((ph & 1) ? 7 - x : x);
  if (l >= T.L) return;
  const int64_t n_chunks = (n_points + kPtsPerBlock - 1) / kPtsPerBlock;
  constexpr int kAtOnce = kEncThreads / kPtsPerBlock;
  for (int64_t c = w + (int64_t)(threadIdx.x / kPtsPerBlock) * G; c < n_chunks; c += (int64_t)kAtOnce * G) {
    const int64_t p = c * kPtsPerBlock + (threadIdx.x % kPtsPerBlock);
    if (p >= n_points) continue;
    const int64_t ray = p / N;
    const RayRec rr = rays[ray];
    float x[3] = {0.0f, 0.0f, 0.0f};
    if (rr.hit) sample_pos(g, rr, (int)(p - ray * N), u24f(mix32((unsigned)p)), x);
    uint32_t idx[8];
    float w8[8];
    level_corners(T.res[l], T.off[l], T.stride[l], T.mask, x, idx, w8);
    float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      float2 v;
      if constexpr (HALF) v = __half22float2(reinterpret_cast<const __half2*>(table)[idx[k]]);
      else v = reinterpret_cast<const float2*>(table)[idx[k]];
      s0 += w8[k] * v.x;
      s1 += w8[k] * v.y;
    }
    out[(int64_t)l * n_points + p] = make_float2(s0, s1);
  }
}

// The same gathers in a forward kernel's own layout: 4 waves x 32 points per chunk, lane half h
// gathering levels 4j + 2h + q, every level on every XCD; one summed output per point.
template <int L, bool HALF>
__global__ void __launch_bounds__(kBlock, 2) k_encode_only(const LevelTab T, const void* __restrict__ table,
                                                           const RayRec* __restrict__ rays, Geo g, int N,
                                                           int64_t n_points, float* __restrict__ out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, n = lane & 31, h = lane >> 5;
  const int64_t n_chunks = (n_points + kPtsPerBlock - 1) / kPtsPerBlock;
  for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
    const int64_t wave_id = chunk * kWavesPerBlock + wv;
    const int64_t p = wave_id * kPtsPerWave + n;
    if (wave_id * kPtsPerWave >= n_points) continue;
    const int64_t ray = (wave_id * kPtsPerWave) / N;
    const int i = (int)(p - ray * N);
    const RayRec rr = rays[ray];
    float x[3] = {0.0f, 0.0f, 0.0f};
    if (rr.hit) sample_pos(g, rr, i, u24f(mix32((unsigned)p)), x);
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < L / 4; ++j) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int l = 4 * j + 2 * h + q;
        uint32_t idx[8];
        float w[8];
        level_corners(T.res[l], T.off[l], T.stride[l], T.mask, x, idx, w);
        float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          float2 v;
          if constexpr (HALF) v = __half22float2(reinterpret_cast<const __half2*>(table)[idx[c]]);
          else v = reinterpret_cast<const float2*>(table)[idx[c]];
          s0 += w[c] * v.x;
          s1 += w[c] * v.y;
        }
        acc += s0 + s1;
      }
    }
    acc += __shfl_xor(acc, 32, 64);
    if (h == 0 && p < n_points) out[p] = acc;
  }
}

template <typename E>
__device__ __forceinline__ float entry_sum(const E* t, unsigned i);
template <>
__device__ __forceinline__ float entry_sum<float2>(const float2* t, unsigned i) {
  const float2 v = t[i];
  return v.x + v.y;
}
template <>
__device__ __forceinline__ float entry_sum<__half2>(const __half2* t, unsigned i) {
  const float2 v = __half22float2(t[i]);
  return v.x + v.y;
}

// 8 cells per lane, 8 corners per cell: pairs (h, h + 1) of x-adjacent entries.
template <typename E>
__global__ void k_gather(const E* __restrict__ t, unsigned n, float* __restrict__ out, unsigned seed) {
  const unsigned gid = blockIdx.x * blockDim.x + threadIdx.x;
  float acc = 0.0f;
#pragma unroll
  for (int cell = 0; cell < 8; ++cell) {
    const unsigned base = mix32(gid * 8u + cell + seed);
#pragma unroll
    for (int c = 0; c < 8; ++c) acc += entry_sum<E>(t, (mix32(base + (c >> 1)) + (c & 1)) % n);
  }
  out[gid] = acc;
}

__global__ void k_atomic(float* __restrict__ t, unsigned n_entries, unsigned seed) {
  const unsigned gid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int cell = 0; cell < 8; ++cell) {
    const unsigned base = mix32(gid * 8u + cell + seed);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const unsigned e = (mix32(base + (c >> 1)) + (c & 1)) % n_entries;
      atomicAdd(&t[2 * e], 1e-3f);
      atomicAdd(&t[2 * e + 1], 1e-3f);
    }
  }
}

__global__ void k_records(const BinRec* __restrict__ r, unsigned n, float* __restrict__ out) {
  const unsigned stride = gridDim.x * blockDim.x;
  float acc = 0.0f;
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const BinRec x = r[i];
    acc += x.v0 + x.v1 + (float)(x.idx & 1u);
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

template <int MODE>
__global__ void __launch_bounds__(1024) k_lds(float* __restrict__ out, int iters) {
  constexpr int kWords = 8192;   // 64 KB as u64
  __shared__ unsigned long long s64[kWords];
  float* sf = reinterpret_cast<float*>(s64);
  unsigned* su = reinterpret_cast<unsigned*>(s64);
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) s64[i] = 0ull;
  __syncthreads();
  unsigned h = mix32(blockIdx.x * 1024u + threadIdx.x);
  for (int it = 0; it < iters; ++it) {
    h = mix32(h + it);
    const unsigned w = h & (kWords - 1);
    if (MODE == 0) atomicAdd(&sf[w], 1.0f);
    if (MODE == 1) atomicAdd(&su[w], 1u);
    if (MODE == 2) atomicAdd(&s64[w], 1ull);
  }
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = sf[0] + (float)su[1] + (float)s64[2];
}

struct Timer {
  hipEvent_t a, b;
  Timer() {
    UB_CHECK(hipEventCreate(&a));
    UB_CHECK(hipEventCreate(&b));
  }
  void start() { UB_CHECK(hipEventRecord(a)); }
  float stop_ms() {
    UB_CHECK(hipEventRecord(b));
    UB_CHECK(hipEventSynchronize(b));
    float ms = 0.0f;
    UB_CHECK(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
};

constexpr int kReps = 5;

// Best of several grid sizes (256 threads per block) for a launch of f(blocks); returns ms per launch.
template <typename F>
float best_grid(Timer& tm, F f, int& best_blocks) {
  const int grids[] = {1024, 2048, 4096, 8192, 16384, 32768};
  float best = 1e30f;
  for (int blocks : grids) {
    f(blocks);
    tm.start();
    for (int r = 0; r < kReps; ++r) f(blocks);
    const float ms = tm.stop_ms() / kReps;
    if (ms < best) {
      best = ms;
      best_blocks = blocks;
    }
  }
  return best;
}

void streams(Timer& tm) {
  const size_t bytes = 1ull << 30, n = bytes / 16;
  float4 *a, *b;
  float* out;
  UB_CHECK(hipMalloc(&a, bytes));
  UB_CHECK(hipMalloc(&b, bytes));
  UB_CHECK(hipMalloc(&out, 64));
  UB_CHECK(hipMemset(a, 0, bytes));
  UB_CHECK(hipMemset(b, 0, bytes));
  int bb = 0;
  float ms = best_grid(tm, [&](int blocks) { k_stream_copy<<<blocks, 256>>>(a, b, n); }, bb);
  std::printf("stream_copy 1 GiB: %.0f GB/s (read + write; best grid %d x 256)\n", 2.0 * bytes / (ms * 1e-3) / 1e9, bb);
  std::printf("ceiling stream_copy %.1f GB/s\n", 2.0 * bytes / (ms * 1e-3) / 1e9);
  ms = best_grid(tm, [&](int blocks) { k_stream_read<<<blocks, 256>>>(a, n, out); }, bb);
  std::printf("stream_read 1 GiB: %.0f GB/s (best grid %d x 256)\n", bytes / (ms * 1e-3) / 1e9, bb);
  std::printf("ceiling stream_read %.1f GB/s\n", bytes / (ms * 1e-3) / 1e9);
  ms = best_grid(tm, [&](int blocks) { k_stream_write<<<blocks, 256>>>(b, n, 1.0f); }, bb);
  std::printf("stream_write 1 GiB: %.0f GB/s (best grid %d x 256)\n", bytes / (ms * 1e-3) / 1e9, bb);
  std::printf("ceiling stream_write %.1f GB/s\n", bytes / (ms * 1e-3) / 1e9);
  const size_t n2 = (2ull << 20) / 16;
  const int reps = 256;
  k_copy_l2<<<1024, 256>>>(a, b, n2, reps);
  tm.start();
  for (int r = 0; r < kReps; ++r) k_copy_l2<<<1024, 256>>>(a, b, n2, reps);
  ms = tm.stop_ms() / kReps;
  std::printf("copy_l2 2 MiB x %d: %.0f GB/s (read + write)\n", reps, 2.0 * 16 * n2 * reps / (ms * 1e-3) / 1e9);
  UB_CHECK(hipFree(a));
  UB_CHECK(hipFree(b));
  UB_CHECK(hipFree(out));
}

// The 256^3 workload's encoder (16 levels x 2 features, T = 2^19, N_min 16, N_max 2048) and one
// view of 2048 rays x 192 samples.
void encode_ceiling(Timer& tm) {
  constexpr int L = 16;
  const int R = 2048, N = 192, n_det = 256, n_cu_blocks_per = 2;
  const double b = std::exp((std::log(2048.0) - std::log(16.0)) / (L - 1));
  const uint64_t T = 1ull << 19;
  LevelTab lt{};
  uint64_t off = 0;
  for (int l = 0; l < L; ++l) {
    const int32_t Nl = (int32_t)std::floor(16.0 * std::pow(b, (double)l));
    const double nv = ((double)Nl + 1.0) * ((double)Nl + 1.0) * ((double)Nl + 1.0);
    const bool dense = nv <= (double)T;
    lt.res[l] = Nl;
    lt.off[l] = (uint32_t)off;
    lt.stride[l] = dense ? (uint32_t)(Nl + 1) : 0u;
    off += dense ? (uint64_t)nv : T;
  }
  lt.mask = (uint32_t)(T - 1);
  lt.L = L;
  lt.on = 0xFFFFFFFFu;
  lt.bin_shift = 13;
  const uint64_t n_entries = off;
  Geo g{};
  g.dso = 1000.0;
  g.back = 500.0;
  g.du = g.dv = 384.0 / n_det;
  g.nu = g.nv = n_det;
  for (int k = 0; k < 3; ++k) {
    g.vol[k] = 256.0;
    g.inv_vol[k] = 1.0 / 256.0;
  }
  const double th = 2.0 * 3.14159265358979323846 * 17.0 / 50.0;
  RayRec* rays;
  float* out;
  void* table;
  const int64_t P = (int64_t)R * N;
  UB_CHECK(hipMalloc(&rays, sizeof(RayRec) * R));
  UB_CHECK(hipMalloc(&out, sizeof(float2) * P * L));
  UB_CHECK(hipMalloc(&table, n_entries * 8));
  UB_CHECK(hipMemset(table, 0, n_entries * 8));
  k_ub_rays<<<(R + 255) / 256, 256>>>(g, std::cos(th), std::sin(th), R, n_det * n_det, N, rays);
  int dev = 0, n_cu = 0;
  UB_CHECK(hipGetDevice(&dev));
  UB_CHECK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  const int grid = n_cu * n_cu_blocks_per;   // the backward grid of the step: point groups
  const double gathers = (double)P * L * 8;
  for (int lanes = 0; lanes < 2; ++lanes) {
    for (int half = 0; half < 2; ++half) {
      auto launch = [&]() {
        if (lanes) {
          if (half) k_encode_only<L, true><<<grid, kBlock>>>(lt, table, rays, g, N, P, out);
          else k_encode_only<L, false><<<grid, kBlock>>>(lt, table, rays, g, N, P, out);
        } else {
          const unsigned blocks = 8u * ((L + 7) / 8) * (unsigned)grid;
          float2* o2 = reinterpret_cast<float2*>(out);
          if (half) k_encode_lvl<true><<<blocks, kEncThreads>>>(lt, table, rays, g, N, P, grid, o2);
          else k_encode_lvl<false><<<blocks, kEncThreads>>>(lt, table, rays, g, N, P, grid, o2);
        }
      };
      launch();
      tm.start();
      for (int r = 0; r < 4 * kReps; ++r) launch();
      const float ms = tm.stop_ms() / (4 * kReps);
      const char* nm = lanes ? (half ? "encode_lanes_fp16" : "encode_lanes_fp32") : (half ? "encode_fp16" : "encode_fp32");
      std::printf("%s 256^3 workload (%lld points x 16 levels x 8 corners, table %.1f MB): %.1f us per step, "
                  "%.1f G gathers/s\n", nm, (long long)P, n_entries * (half ? 4.0 : 8.0) / 1e6, ms * 1e3,
                  gathers / (ms * 1e-3) / 1e9);
      if (!lanes) std::printf("ceiling %s %.2f us\n", nm, ms * 1e3);
    }
  }
  UB_CHECK(hipFree(rays));
  UB_CHECK(hipFree(out));
  UB_CHECK(hipFree(table));
}

void random_patterns(Timer& tm) {
  const unsigned lanes = 1u << 22;
  float* out;
  UB_CHECK(hipMalloc(&out, (size_t)lanes * 4));
  const double table_mb[] = {0.94, 48.8, 169.0};
  for (double mb : table_mb) {   // gathers and spread atomics
    const unsigned n = (unsigned)(mb * 1e6 / 8);
    void* t;
    UB_CHECK(hipMalloc(&t, (size_t)n * 8));
    UB_CHECK(hipMemset(t, 0, (size_t)n * 8));
    const double gathers = (double)lanes * 64 * kReps;
    k_gather<float2><<<lanes / 256, 256>>>((const float2*)t, n, out, 1);
    tm.start();
    for (int r = 0; r < kReps; ++r) k_gather<float2><<<lanes / 256, 256>>>((const float2*)t, n, out, r);
    float ms = tm.stop_ms();
    std::printf("gather_fp32x2 table %.2f MB: %.1f G gathers/s\n", mb, gathers / (ms * 1e-3) / 1e9);
    const unsigned n16 = (unsigned)(mb * 1e6 / 8);   // same entry count, half the bytes
    k_gather<__half2><<<lanes / 256, 256>>>((const __half2*)t, n16, out, 1);
    tm.start();
    for (int r = 0; r < kReps; ++r) k_gather<__half2><<<lanes / 256, 256>>>((const __half2*)t, n16, out, r);
    ms = tm.stop_ms();
    std::printf("gather_fp16x2 table %.2f MB: %.1f G gathers/s\n", mb / 2, gathers / (ms * 1e-3) / 1e9);
    if (mb > 10.0 && mb < 100.0) {
      k_atomic<<<lanes / 256, 256>>>((float*)t, n, 1);
      tm.start();
      for (int r = 0; r < kReps; ++r) k_atomic<<<lanes / 256, 256>>>((float*)t, n, r);
      ms = tm.stop_ms();
      std::printf("atomic_f32 spread table %.2f MB: %.1f G atomics/s\n", mb, 2 * gathers / (ms * 1e-3) / 1e9);
    }
    UB_CHECK(hipFree(t));
  }
  {  // contended atomics: 4913 entries x 2 floats
    const unsigned n = 4913;
    float* t;
    UB_CHECK(hipMalloc(&t, (size_t)n * 8));
    UB_CHECK(hipMemset(t, 0, (size_t)n * 8));
    k_atomic<<<lanes / 256, 256>>>(t, n, 1);
    tm.start();
    for (int r = 0; r < kReps; ++r) k_atomic<<<lanes / 256, 256>>>(t, n, r);
    const float ms = tm.stop_ms();
    std::printf("atomic_f32 contended 4913 entries: %.1f G atomics/s\n",
                (double)lanes * 128 * kReps / (ms * 1e-3) / 1e9);
    UB_CHECK(hipFree(t));
  }
  {  // record stream
    const unsigned n = 33u << 20;
    BinRec* r;
    UB_CHECK(hipMalloc(&r, (size_t)n * sizeof(BinRec)));
    UB_CHECK(hipMemset(r, 0, (size_t)n * sizeof(BinRec)));
    k_records<<<2048, 256>>>(r, n, out);
    tm.start();
    for (int k = 0; k < kReps; ++k) k_records<<<2048, 256>>>(r, n, out);
    const float ms = tm.stop_ms();
    std::printf("records 12 B x %u: %.0f GB/s\n", n, (double)n * sizeof(BinRec) * kReps / (ms * 1e-3) / 1e9);
    UB_CHECK(hipFree(r));
  }
  {  // LDS atomics
    const int blocks = 512, iters = 2048;
    const double ops = (double)blocks * 1024 * iters * kReps;
    const char* names[3] = {"lds_add_f32", "lds_add_u32", "lds_add_u64"};
    for (int mode = 0; mode < 3; ++mode) {
      auto launch = [&]() {
        if (mode == 0) k_lds<0><<<blocks, 1024>>>(out, iters);
        if (mode == 1) k_lds<1><<<blocks, 1024>>>(out, iters);
        if (mode == 2) k_lds<2><<<blocks, 1024>>>(out, iters);
      };
      launch();
      tm.start();
      for (int r = 0; r < kReps; ++r) launch();
      const float ms = tm.stop_ms();
      std::printf("%s random 64 KB: %.0f G lane-atomics/s\n", names[mode], ops / (ms * 1e-3) / 1e9);
    }
  }
  UB_CHECK(hipFree(out));
}

}  // namespace

int main(int argc, char** argv) {
  const bool quick = argc > 1 && std::strcmp(argv[1], "--quick") == 0;
  Timer tm;
  streams(tm);
  encode_ceiling(tm);
  if (!quick) random_patterns(tm);
  UB_CHECK(hipGetLastError());
  UB_CHECK(hipDeviceSynchronize());
  std::printf("ubench done\n");
  return 0;
}
