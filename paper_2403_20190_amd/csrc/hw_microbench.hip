// hw_microbench.hip -- probes of the device's peak rates, used to price the
// roofline of the hot-path kernels against what this GPU delivers: a stream
// triad for HBM bandwidth, and the issue rate of the 32-bit VALU instructions
// the modular arithmetic is made of (v_add_u32, v_mul_lo_u32, v_mul_hi_u32,
// v_mad_u64_u32) at full occupancy.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>

#include "../../include/hwisard.h"
#include "hw_ctx.h"

namespace {

// a[i] = b[i] + k c[i] over n uint4 words (uint32 lanes, wrapping)
__global__ __launch_bounds__(256) void k_triad(uint4* __restrict__ a, const uint4* __restrict__ b,
                                               const uint4* __restrict__ c, uint32_t k, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint4 x = b[i], y = c[i];
    a[i] = make_uint4(x.x + k * y.x, x.y + k * y.y, x.z + k * y.z, x.w + k * y.w);
  }
}

__global__ __launch_bounds__(256) void k_fill(uint4* __restrict__ a, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = make_uint4(v, v + 1, v + 2, v + 3);
}

constexpr int CHAINS = 8, UNROLL = 16;

// OP: 0 v_add_u32, 1 v_mul_lo_u32, 2 v_mul_hi_u32, 3 v_mad_u64_u32.  Each
// thread runs CHAINS independent dependency chains of the instruction,
// UNROLL deep per loop trip; a result no input can produce is the only
// store, which keeps every chain live.
template <int OP>
__global__ __launch_bounds__(256) void k_valu(uint32_t iters, uint32_t* out) {
  const uint32_t m = 0x9E3779B9u ^ (threadIdx.x * 2654435761u);
  uint32_t a[CHAINS];
  uint64_t w[CHAINS];
#pragma unroll
  for (int k = 0; k < CHAINS; ++k) {
    a[k] = threadIdx.x + 977u * k + 1u;
    w[k] = a[k];
  }
#pragma unroll 1
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < UNROLL; ++r)
#pragma unroll
      for (int k = 0; k < CHAINS; ++k) {
        if constexpr (OP == 0) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(m));
        else if constexpr (OP == 1) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[k]) : "v"(m));
        else if constexpr (OP == 2) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[k]) : "v"(m));
        else {
          uint64_t d, carry;
          asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(d), "=s"(carry) : "v"(a[k]), "v"(m), "v"(w[k]));
          w[k] = d;
        }
      }
  }
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < CHAINS; ++k) x ^= a[k] ^ (uint32_t)w[k] ^ (uint32_t)(w[k] >> 32);
  if (x == 0xFFFFFFFFu && m == 0u) out[0] = x;  // m is never 0 for threadIdx.x < 256
}

template <class F>
hipError_t best_ms(hipStream_t st, int reps, F&& launch, float* best) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  *best = 1e30f;
  for (int r = 0; e == hipSuccess && r < reps; ++r) {
    e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess && ms < *best) *best = ms;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return e;
}

}  // namespace

extern "C" hw_status hw_microbench(int device, const char* kind, uint64_t size, double* rate, double* ms,
                                   hipStream_t st) {
  if (!kind || !rate) return fail(HW_EINVAL, "null argument");
  HIP_TRY(hipSetDevice(device));
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  float best = 0;
  if (!strcmp(kind, "triad")) {
    const uint64_t words = size / 16;  // uint4 per array
    if (words < 1024) return fail(HW_EINVAL, "triad arrays of %llu bytes: at least 16 KiB",
                                  (unsigned long long)size);
    uint4* buf = nullptr;
    HIP_TRY(hipMalloc(&buf, 3 * words * 16));
    uint4 *a = buf, *b = buf + words, *c = buf + 2 * words;
    const uint32_t grid = (uint32_t)cus * 16;
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, st, b, words, 1u);
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, st, c, words, 7u);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = best_ms(st, 5, [&] {
        hipLaunchKernelGGL(k_triad, dim3(grid), dim3(256), 0, st, a, b, c, 3u, words);
        return hipGetLastError();
      }, &best);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    HIP_TRY(e);
    *rate = 3.0 * words * 16 / (best / 1000.0);  // bytes/s: two arrays read, one written
  } else {
    int op = -1;
    const char* names[4] = {"v_add_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mad_u64_u32"};
    for (int i = 0; i < 4; ++i)
      if (!strcmp(kind, names[i])) op = i;
    if (op < 0) return fail(HW_EINVAL, "unknown probe '%s'", kind);
    const uint32_t iters = size ? (uint32_t)size : 4096u;
    const uint32_t grid = (uint32_t)cus * 8;  // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    uint32_t* out = nullptr;
    HIP_TRY(hipMalloc(&out, 64));
    hipError_t e = best_ms(st, 3, [&] {
      switch (op) {
        case 0: hipLaunchKernelGGL(k_valu<0>, dim3(grid), dim3(256), 0, st, iters, out); break;
        case 1: hipLaunchKernelGGL(k_valu<1>, dim3(grid), dim3(256), 0, st, iters, out); break;
        case 2: hipLaunchKernelGGL(k_valu<2>, dim3(grid), dim3(256), 0, st, iters, out); break;
        default: hipLaunchKernelGGL(k_valu<3>, dim3(grid), dim3(256), 0, st, iters, out); break;
      }
      return hipGetLastError();
    }, &best);
    (void)hipStreamSynchronize(st);
    (void)hipFree(out);
    HIP_TRY(e);
    *rate = (double)grid * 256 * iters * UNROLL * CHAINS / (best / 1000.0);  // lane-instructions/s
  }
  if (ms) *ms = best;
  return ok();
}
