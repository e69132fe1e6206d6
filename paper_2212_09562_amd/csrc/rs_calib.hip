// VALU issue-rate calibration for the integer roofline.
//
// The construction is bound by integer vector-ALU issue: one hash evaluation
// (mixer, reduction to a position, bit update) is a fixed sequence of 32- and
// 64-bit integer instructions.  Each loop below issues one instruction class
// over 8 independent dependency chains per lane at full occupancy, so its
// throughput is the class's issue rate.  The plain 32-bit add sets the
// full-rate reference; the cost of a class in full-rate slots is
// rate(add) / rate(class).  A ninth kernel runs the hash sequence itself
// (keys in registers, no memory) for the attainable evaluation rate.
#include <hip/hip_runtime.h>

#include "rs_launch.h"

namespace rs {

namespace {

constexpr uint32_t kCalThreads = 256;

template <int OP>
__global__ void __launch_bounds__(kCalThreads) k_calib(uint32_t* out, uint32_t iters, uint32_t seed) {
  const uint32_t t = blockIdx.x * kCalThreads + threadIdx.x;
  uint32_t a[8];
  uint64_t w[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = seed * (t + 1) + 0x9E3779B9u * (j + 1);
    w[j] = ((uint64_t)a[j] << 32) | (a[j] ^ 0x5bd1e995u);
  }
  const uint32_t c = seed | 1u;
  const uint64_t c64 = 0xBF58476D1CE4E5B9ull;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (OP == 0) asm volatile("v_add_u32 %0, %1, %2" : "=v"(a[j]) : "v"(a[j]), "v"(c));
      if (OP == 1) asm volatile("v_xor_b32 %0, %1, %2" : "=v"(a[j]) : "v"(a[j]), "v"(c));
      if (OP == 2) asm volatile("v_mul_lo_u32 %0, %1, %2" : "=v"(a[j]) : "v"(a[j]), "v"(c));
      if (OP == 3) asm volatile("v_mul_hi_u32 %0, %1, %2" : "=v"(a[j]) : "v"(a[j]), "v"(c));
      if (OP == 4)
        asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(w[j]) : "v"(a[j]), "v"(c) : "vcc");
      if (OP == 5) asm volatile("v_lshrrev_b64 %0, 27, %1" : "=v"(w[j]) : "v"(w[j]));
      if (OP == 6) asm volatile("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(w[j]) : "v"(w[j]), "v"(c64));
      if (OP == 7) asm volatile("v_add3_u32 %0, %1, %2, %3" : "=v"(a[j]) : "v"(a[j]), "v"(c), "v"(c));
      if (OP == 4) a[j] = (uint32_t)w[j];
    }
  }
  uint64_t r = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) r ^= a[j] ^ w[j];
  out[t] = (uint32_t)r ^ (uint32_t)(r >> 32);
}

// The evaluation sequence of a bijection trial: 16 keys in registers, lane =
// seed, the leaf size a kernel argument (as in the search kernels, so the
// reduction stays a multiply-high and the last xorshift is kept: 19 VALU
// instructions per evaluation, the sequence the roofline counts).
__global__ void __launch_bounds__(kCalThreads) k_calib_hash(uint32_t* out, uint32_t iters,
                                                            uint32_t seed, uint32_t M) {
  const uint32_t t = blockIdx.x * kCalThreads + threadIdx.x;
  uint64_t keys[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) keys[j] = mix64(seed + j);
  uint64_t X = seed + t;
  const uint32_t full = (1u << M) - 1u;
  uint32_t acc = 0;
  for (uint32_t i = 0; i < iters; ++i) {
    uint32_t mask = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) mask |= 1u << reduce(hash_top(keys[j], X), M);
    acc += mask == full;
    X += 1ull << 20;
  }
  out[t] = acc;
}

template <typename K, typename... A>
double time_kernel(K kernel, uint32_t blocks, uint32_t iters, uint32_t* buf, A... extra) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kCalThreads), 0, 0, buf, iters / 8, 12345u,
                     extra...);
  (void)hipEventRecord(e0, 0);
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kCalThreads), 0, 0, buf, iters, 12345u, extra...);
  (void)hipEventRecord(e1, 0);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return hipGetLastError() == hipSuccess ? ms * 1e-3 : -1.0;
}

}  // namespace

}  // namespace rs

extern "C" int rs_calibrate_valu(rs_valu_rates* out) {
  using namespace rs;
  if (!out) return RS_ERR_INVALID_ARG;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return RS_ERR_DEVICE;
  const uint32_t blocks = (uint32_t)cus * 8;  // 8 waves per SIMD
  uint32_t* buf = nullptr;
  if (hipMalloc(&buf, (size_t)blocks * kCalThreads * sizeof(uint32_t)) != hipSuccess) return RS_ERR_OOM;
  // long enough (several milliseconds) that launch and drain are a small part
  const uint32_t iters = 1u << 16;
  const double lanes = (double)blocks * kCalThreads;
  const double per = lanes * iters * 8.0;
  double s[8];
  s[0] = time_kernel(k_calib<0>, blocks, iters, buf);
  s[1] = time_kernel(k_calib<1>, blocks, iters, buf);
  s[2] = time_kernel(k_calib<2>, blocks, iters, buf);
  s[3] = time_kernel(k_calib<3>, blocks, iters, buf);
  s[4] = time_kernel(k_calib<4>, blocks, iters, buf);
  s[5] = time_kernel(k_calib<5>, blocks, iters, buf);
  s[6] = time_kernel(k_calib<6>, blocks, iters, buf);
  s[7] = time_kernel(k_calib<7>, blocks, iters, buf);
  const uint32_t hiters = 2048;
  const double sh = time_kernel(k_calib_hash, blocks, hiters, buf, 16u);
  // the same loop for about two seconds: the clock the chip holds under a
  // sustained full-occupancy integer load
  const double per_iter = sh / hiters;
  uint32_t long_iters = per_iter > 0 ? (uint32_t)(2.0 / per_iter) : 0;
  if (long_iters < hiters) long_iters = hiters;
  const double sl = time_kernel(k_calib_hash, blocks, long_iters, buf, 16u);
  (void)hipFree(buf);
  for (double v : s)
    if (v <= 0) return RS_ERR_DEVICE;
  if (sh <= 0 || sl <= 0) return RS_ERR_DEVICE;
  out->add_u32 = per / s[0];
  out->xor_b32 = per / s[1];
  out->mul_lo_u32 = per / s[2];
  out->mul_hi_u32 = per / s[3];
  out->mad_u64_u32 = per / s[4];
  out->lshrrev_b64 = per / s[5];
  out->lshl_add_u64 = per / s[6];
  out->add3_u32 = per / s[7];
  out->hash_evals = lanes * hiters * 16.0 / sh;
  out->hash_evals_sustained = lanes * (double)long_iters * 16.0 / sl;
  out->compute_units = (uint32_t)cus;
  return RS_OK;
}
