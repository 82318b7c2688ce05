// Ceilings of the memory access patterns of the training step on one MI355X (gfx950), each timed
// with HIP events over repeated launches after a warm-up launch:
//   copy_hbm      float4 stream copy of 1 GiB (read + write bytes)
//   copy_l2       float4 copy within a 2 MiB buffer, repeated inside the kernel (L2-resident)
//   gather_*      random 8-corner cells (four x-adjacent entry pairs, as at a hash-grid level) of
//                 8-B (FP32 x 2) or 4-B (FP16 x 2) entries in tables of 0.94, 48.8 and 169 MB
//   atomic_*      two global f32 atomic adds per corner, spread over a 48.8 MB table or contended
//                 into 4913 entries (the coarsest level)
//   records       streaming read of 33 M 12-byte records (entry, value, value) as the bin reduction
//                 reads them
//   lds_*         random LDS atomic adds (f32, u32, u64) within a 64 KB block-local array
// Every index is reduced into its buffer before use.  Prints one line per measurement.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define UB_CHECK(x)                                                              \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                              \
    }                                                                            \
  } while (0)

namespace {

__device__ __forceinline__ unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__global__ void k_copy(const float4* __restrict__ a, float4* __restrict__ b, size_t n, size_t total) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += stride) b[i % n] = a[i % n];
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

struct Rec {
  unsigned idx;
  float v0, v1;
};

__global__ void k_records(const Rec* __restrict__ r, unsigned n, float* __restrict__ out) {
  const unsigned stride = gridDim.x * blockDim.x;
  float acc = 0.0f;
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const Rec x = r[i];
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

}  // namespace

int main() {
  Timer tm;
  constexpr int kReps = 5;

  {  // copies
    const size_t bytes = 1ull << 30, n = bytes / 16;
    float4 *a, *b;
    UB_CHECK(hipMalloc(&a, bytes));
    UB_CHECK(hipMalloc(&b, bytes));
    UB_CHECK(hipMemset(a, 0, bytes));
    k_copy<<<8192, 256>>>(a, b, n, n);
    tm.start();
    for (int r = 0; r < kReps; ++r) k_copy<<<8192, 256>>>(a, b, n, n);
    float ms = tm.stop_ms();
    std::printf("copy_hbm 1 GiB: %.0f GB/s (read + write)\n", 2.0 * bytes * kReps / (ms * 1e-3) / 1e9);
    const size_t n2 = (2ull << 20) / 16, total2 = n2 * 256;
    k_copy<<<8192, 256>>>(a, b, n2, total2);
    tm.start();
    for (int r = 0; r < kReps; ++r) k_copy<<<8192, 256>>>(a, b, n2, total2);
    ms = tm.stop_ms();
    std::printf("copy_l2 2 MiB x 256: %.0f GB/s (read + write)\n", 2.0 * 16 * total2 * kReps / (ms * 1e-3) / 1e9);
    UB_CHECK(hipFree(a));
    UB_CHECK(hipFree(b));
  }

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
    Rec* r;
    UB_CHECK(hipMalloc(&r, (size_t)n * sizeof(Rec)));
    UB_CHECK(hipMemset(r, 0, (size_t)n * sizeof(Rec)));
    k_records<<<2048, 256>>>(r, n, out);
    tm.start();
    for (int k = 0; k < kReps; ++k) k_records<<<2048, 256>>>(r, n, out);
    const float ms = tm.stop_ms();
    std::printf("records 12 B x %u: %.0f GB/s\n", n, (double)n * sizeof(Rec) * kReps / (ms * 1e-3) / 1e9);
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
  UB_CHECK(hipGetLastError());
  UB_CHECK(hipFree(out));
  std::printf("ubench done\n");
  return 0;
}
