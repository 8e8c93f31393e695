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

}  // namespace
}  // namespace ising

using namespace ising;

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
