// calibrate.hip -- issue rates of the integer VALU instructions the anneal
// kernels are built from, measured on the current device.  A measurement
// helper for the roofline, not part of the method: eight independent
// register-only chains per lane, launched with eight waves per SIMD, one
// store per lane at the end.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising.h"
#include "runtime.h"

namespace ising {
namespace {

constexpr int kChains = 8;
constexpr int kIters = 4096;
constexpr int kThreads = 256;

// kind: 0 v_mad_u64_u32, 1 v_mul_lo_u32, 2 v_mul_hi_u32, 3 v_xor_b32.
// Each instruction is written out so that the measured opcode is exact.
template <int KIND>
__global__ void __launch_bounds__(kThreads) k_rate(uint32_t* out, uint32_t c) {
  uint32_t lo[kChains], hi[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    lo[j] = threadIdx.x + 977u * (uint32_t)j;
    hi[j] = (uint32_t)j;
  }
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
      if (KIND == 0) {
        uint64_t acc = ((uint64_t)hi[j] << 32) | lo[j];
        asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(acc) : "v"(lo[j]), "s"(c) : "vcc");
        lo[j] = (uint32_t)acc;
        hi[j] = (uint32_t)(acc >> 32);
      } else if (KIND == 1) {
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(lo[j]) : "s"(c));
      } else if (KIND == 2) {
        asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(lo[j]) : "s"(c));
      } else {
        asm volatile("v_xor_b32 %0, %1, %0" : "+v"(lo[j]) : "s"(c));
      }
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s ^= lo[j] ^ hi[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int KIND>
int time_rate(uint32_t* buf, int blocks, hipEvent_t a, hipEvent_t b, double* rate) {
  hipLaunchKernelGGL(k_rate<KIND>, dim3(blocks), dim3(kThreads), 0, nullptr, buf, 0xD2511F53u);
  ICHK(hipEventRecord(a, nullptr));
  hipLaunchKernelGGL(k_rate<KIND>, dim3(blocks), dim3(kThreads), 0, nullptr, buf, 0xD2511F53u);
  ICHK(hipEventRecord(b, nullptr));
  ICHK(hipEventSynchronize(b));
  float ms = 0;
  ICHK(hipEventElapsedTime(&ms, a, b));
  if (ms <= 0) {
    set_error("calibration kernel timed at zero");
    return ISING_ERR_DEVICE;
  }
  *rate = (double)blocks * kThreads * kIters * kChains / (ms * 1e-3);
  return ISING_OK;
}

// LDS read bandwidth: every lane reads 16 bytes per step (ds_read_b128) at
// addresses that put a wave's 64 reads on consecutive 16-byte chunks (no
// bank conflicts), walking a 32 KiB buffer; four workgroups per CU.
constexpr int kLdsThreads = 256;
constexpr int kLdsWords = 32 * 1024 / 4;
constexpr int kLdsIters = 8192;

typedef uint32_t lds_u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kLdsThreads) k_lds_rate(uint32_t* out) {
  __shared__ __align__(16) uint32_t buf[kLdsWords];
  for (int i = threadIdx.x; i < kLdsWords; i += kLdsThreads) buf[i] = (uint32_t)i * 2654435761u;
  __syncthreads();
  // eight reads 4 KiB apart, issued together and waited for in the same
  // block (the compiler would otherwise keep loop-invariant reads out of
  // the loop); lane i reads bytes 16 i .. 16 i + 15 of each 4 KiB
  const uint32_t addr = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t*)buf +
                        16u * threadIdx.x;
  uint32_t acc = 0;
  for (int it = 0; it < kLdsIters / 8; ++it) {
    lds_u32x4 v0, v1, v2, v3, v4, v5, v6, v7;
    asm volatile(
        "ds_read_b128 %0, %8\n\t"
        "ds_read_b128 %1, %8 offset:4096\n\t"
        "ds_read_b128 %2, %8 offset:8192\n\t"
        "ds_read_b128 %3, %8 offset:12288\n\t"
        "ds_read_b128 %4, %8 offset:16384\n\t"
        "ds_read_b128 %5, %8 offset:20480\n\t"
        "ds_read_b128 %6, %8 offset:24576\n\t"
        "ds_read_b128 %7, %8 offset:28672\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=v"(v0), "=v"(v1), "=v"(v2), "=v"(v3), "=v"(v4), "=v"(v5), "=v"(v6), "=v"(v7)
        : "v"(addr));
    acc ^= v0.x ^ v1.y ^ v2.z ^ v3.w ^ v4.x ^ v5.y ^ v6.z ^ v7.w;
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace
}  // namespace ising

using namespace ising;

extern "C" int ising_lds_rate(double* bytes_per_s) {
  if (!bytes_per_s) return ISING_ERR_INVALID;
  int dev = 0, cus = 0;
  ICHK(hipGetDevice(&dev));
  ICHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = std::max(cus, 1) * 4;
  uint32_t* buf = nullptr;
  ICHK(hipMalloc(&buf, sizeof(uint32_t) * (size_t)blocks * kLdsThreads));
  hipEvent_t a = nullptr, b = nullptr;
  int st = ISING_OK;
  float ms = 0;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipEventCreate failed");
    st = ISING_ERR_DEVICE;
  }
  if (st == ISING_OK) {
    hipLaunchKernelGGL(k_lds_rate, dim3(blocks), dim3(kLdsThreads), 0, nullptr, buf);
    if (hipEventRecord(a, nullptr) != hipSuccess) st = ISING_ERR_DEVICE;
    hipLaunchKernelGGL(k_lds_rate, dim3(blocks), dim3(kLdsThreads), 0, nullptr, buf);
    if (st == ISING_OK && (hipEventRecord(b, nullptr) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                           hipEventElapsedTime(&ms, a, b) != hipSuccess))
      st = ISING_ERR_DEVICE;
    if (st != ISING_OK) {
      (void)hipGetLastError();
      set_error("LDS rate kernel failed");
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(buf);
  if (st != ISING_OK) return st;
  if (ms <= 0) {
    set_error("LDS rate kernel timed at zero");
    return ISING_ERR_DEVICE;
  }
  *bytes_per_s = (double)blocks * kLdsThreads * kLdsIters * 16.0 / (ms * 1e-3);
  return ISING_OK;
}

extern "C" int ising_valu_rates(double* rates) {
  if (!rates) return ISING_ERR_INVALID;
  int dev = 0, cus = 0;
  ICHK(hipGetDevice(&dev));
  ICHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = std::max(cus, 1) * 8;  // eight 64-lane waves per SIMD
  uint32_t* buf = nullptr;
  ICHK(hipMalloc(&buf, sizeof(uint32_t) * (size_t)blocks * kThreads));
  hipEvent_t a = nullptr, b = nullptr;
  int st = ISING_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipEventCreate failed");
    st = ISING_ERR_DEVICE;
  }
  double r[4] = {0, 0, 0, 0};
  if (st == ISING_OK) st = time_rate<0>(buf, blocks, a, b, &r[0]);
  if (st == ISING_OK) st = time_rate<1>(buf, blocks, a, b, &r[1]);
  if (st == ISING_OK) st = time_rate<2>(buf, blocks, a, b, &r[2]);
  if (st == ISING_OK) st = time_rate<3>(buf, blocks, a, b, &r[3]);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(buf);
  if (st != ISING_OK) return st;
  for (int i = 0; i < 4; ++i) rates[i] = r[i];
  return ISING_OK;
}
