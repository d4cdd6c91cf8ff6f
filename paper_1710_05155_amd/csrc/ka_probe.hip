// ka_probe.hip -- microbenchmarks of the integer vector ALU (gfx950), for the roofline of the
// bit-logic kernels: the issue rate of plain 32-bit bitwise instructions and of the 32 x 32 ->
// 64-bit multiply-add that Philox4x32 rounds are built from.  Each thread runs chains of
// register-only instructions written in inline assembly, so the instruction count per launch
// is exact: no memory operand appears in the timed loop.
#include <cstdint>

#include "ka_objects.h"

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeChains = 8;     // independent chains per thread (hides the latency)

// kind 0: v_xor_b32.  Per iteration each of the 8 chains issues 8 instructions: 64 per thread.
__global__ __launch_bounds__(kProbeBlock) void k_probe_xor(uint32_t *out, int iters)
{
  const uint32_t k = (uint32_t)blockIdx.x * 2654435761u + 1u;
  uint32_t a[kProbeChains];
#pragma unroll
  for (int q = 0; q < kProbeChains; ++q) a[q] = (uint32_t)threadIdx.x * (2u * q + 1u) + (uint32_t)q;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
#pragma unroll
      for (int q = 0; q < kProbeChains; ++q) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[q]) : "v"(k));
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int q = 0; q < kProbeChains; ++q) x ^= a[q];
  out[blockIdx.x * kProbeBlock + threadIdx.x] = x;
}

// kind 1: v_mad_u64_u32 (64-bit result of a 32 x 32 product plus a 64-bit addend), with the
// multiplier in a scalar register as in the Philox rounds.  Per iteration each of the 8 chains
// issues 2 instructions: 16 per thread.  The carry-out goes to a scratch scalar pair.
__global__ __launch_bounds__(kProbeBlock) void k_probe_mad(uint64_t *out, int iters)
{
  const uint32_t m = 0xD2511F53u ^ (uint32_t)blockIdx.x;
  uint64_t a[kProbeChains];
#pragma unroll
  for (int q = 0; q < kProbeChains; ++q) a[q] = (uint64_t)threadIdx.x * (2u * q + 3u);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
      for (int q = 0; q < kProbeChains; ++q)
        asm volatile("v_mad_u64_u32 %0, s[40:41], %1, %2, %0"
                     : "+v"(a[q])
                     : "v"((uint32_t)threadIdx.x + (uint32_t)q), "s"(m)
                     : "s40", "s41");
    }
  }
  uint64_t x = 0;
#pragma unroll
  for (int q = 0; q < kProbeChains; ++q) x ^= a[q];
  out[blockIdx.x * kProbeBlock + threadIdx.x] = x;
}

}  // namespace

extern "C" int ka_probe_valu(int kind, int iters, int blocks, void *hip_stream, double *instr_per_s,
                             double *lane_ops_per_s)
{
  return ka_guard([&]() -> int {
    if ((kind != 0 && kind != 1) || iters < 1 || blocks < 1 || blocks > (1 << 20) || !instr_per_s) {
      ka_set_error("ka_probe_valu: kind must be 0 or 1, iters >= 1, blocks in [1, 2^20]");
      return KA_EINVAL;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    bool own = false;
    if (!s) {
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        ka_set_error("ka_probe_valu: stream creation failed");
        return KA_EDEVICE;
      }
      own = true;
    }
    void *buf = nullptr;
    const size_t n = (size_t)blocks * kProbeBlock;
    hipError_t e = hipMalloc(&buf, n * sizeof(uint64_t));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0.f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // the first launch is a warm-up
      e = hipEventRecord(e0, s);
      if (e == hipSuccess) {
        if (kind == 0)
          hipLaunchKernelGGL(k_probe_xor, dim3((unsigned)blocks), dim3(kProbeBlock), 0, s, (uint32_t *)buf, iters);
        else
          hipLaunchKernelGGL(k_probe_mad, dim3((unsigned)blocks), dim3(kProbeBlock), 0, s, (uint64_t *)buf, iters);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamSynchronize(s);
    if (buf) (void)hipFree(buf);
    if (own) (void)hipStreamDestroy(s);
    if (e != hipSuccess || ms <= 0.f) {
      ka_set_error(e != hipSuccess ? hipGetErrorString(e) : "ka_probe_valu: no elapsed time");
      return KA_EDEVICE;
    }
    const double per_thread = (double)iters * (kind == 0 ? 64.0 : 16.0);
    const double waves = (double)blocks * (kProbeBlock / 64);
    *instr_per_s = waves * per_thread / (ms * 1e-3);
    if (lane_ops_per_s) *lane_ops_per_s = *instr_per_s * 64.0;
    return KA_OK;
  });
}
