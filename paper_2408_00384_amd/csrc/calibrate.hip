// Roofline calibration: the LDS read bandwidth and the 32-bit VALU issue rate
// this device reaches, measured rather than taken from a data sheet, for the
// LDS-resident batched kernel's roofline.  Not part of the simulation path.
//
//   k_cal_lds:  every lane reads 16 bytes per LDS instruction, consecutive
//               lanes at consecutive addresses (no bank conflicts), 8 reads
//               in flight per iteration, 8 workgroups of 256 threads per CU.
//   k_cal_valu: 8 independent chains of v_xor_b32 per lane (written as
//               inline VALU instructions so the compiler can neither merge
//               them into three-input ops nor drop them).
#include "internal.h"

namespace cliff {

constexpr uint32_t kCalThreads = 256;
constexpr uint32_t kCalLdsVec = 2048;   // 32 KB of uint4 (the 8 reads of an iteration are distinct)
constexpr uint32_t kCalLdsUnroll = 8;
constexpr uint32_t kCalValuChains = 8, kCalValuUnroll = 16;

__global__ void __launch_bounds__(kCalThreads) k_cal_lds(uint32_t iters, uint32_t *sink) {
  __shared__ uint4 buf[kCalLdsVec];
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < kCalLdsVec; i += kCalThreads) buf[i] = make_uint4(i, 3 * i + 1, 5 * i + 2, 7 * i + 3);
  __syncthreads();
  uint4 acc = make_uint4(0, 0, 0, 0);
  uint32_t base = tid;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (uint32_t u = 0; u < kCalLdsUnroll; ++u) {
      const uint4 v = buf[(base + u * kCalThreads) & (kCalLdsVec - 1)];
      acc.x ^= v.x;
      acc.y ^= v.y;
      acc.z ^= v.z;
      acc.w ^= v.w;
    }
    base = (base + 64) & (kCalLdsVec - 1);
  }
  // practically never true; keeps every read live
  if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x9e3779b9u) sink[blockIdx.x % 1024] = acc.x;
}

__global__ void __launch_bounds__(kCalThreads) k_cal_valu(uint32_t iters, uint32_t *sink) {
  uint32_t a[kCalValuChains], k[kCalValuChains];
#pragma unroll
  for (uint32_t c = 0; c < kCalValuChains; ++c) {
    a[c] = threadIdx.x * (c + 1);
    k[c] = blockIdx.x + 0x01000193u * (c + 1);
  }
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (uint32_t u = 0; u < kCalValuUnroll; ++u) {
#pragma unroll
      for (uint32_t c = 0; c < kCalValuChains; ++c) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[c]) : "v"(k[c]));
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (uint32_t c = 0; c < kCalValuChains; ++c) x ^= a[c];
  if (x == 0x9e3779b9u) sink[blockIdx.x % 1024] = x;
}

// kind 0: LDS bytes, 1: VALU 32-bit lane operations, per launch in *work.
// sink: 1024 device words (written only by an improbable branch).
hipError_t launch_calibrate(int kind, int num_cus, uint32_t iters, uint32_t *sink, hipStream_t st, double *work) {
  const uint32_t grid = uint32_t(num_cus) * 8;
  if (kind == 0) {
    k_cal_lds<<<grid, kCalThreads, 0, st>>>(iters, sink);
    *work = double(grid) * kCalThreads * iters * kCalLdsUnroll * 16.0;
  } else {
    k_cal_valu<<<grid, kCalThreads, 0, st>>>(iters, sink);
    *work = double(grid) * kCalThreads * iters * kCalValuUnroll * kCalValuChains;
  }
  return hipGetLastError();
}

}  // namespace cliff
