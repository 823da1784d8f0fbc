// Measured 32-bit VALU issue rate of the device, reported beside the nominal
// peak the pair kernel's roofline fraction is taken against.
//
// Every wave runs eight independent dependency chains of v_xor_b32 /
// v_add_u32 (plain 32-bit VALU instructions, the kind the Myers/Hyyro step
// issues), written as volatile inline assembly so that the compiler can
// neither fold nor fuse them.  Eight waves per SIMD keep every SIMD's issue
// ports busy: on gfx950 two waves of a SIMD can issue instructions of this
// class in the same 4-clock window, so the nominal rate of the class is
// CUs x 128 lanes x clock (the FP32 FMA vector rate, in instructions).
#define TCRNET_BUILDING 1
#include <algorithm>

#include "api_internal.h"

namespace {

constexpr uint32_t kPerIter = 8 * 16;  // instructions per loop iteration

// One inline-assembly block per round: 8 xors then 8 adds on 8 chains.
#define TCR_PROBE_ROUND                                                                                   \
  asm volatile(                                                                                           \
      "v_xor_b32 %0, %0, %8\n v_xor_b32 %1, %1, %8\n v_xor_b32 %2, %2, %8\n v_xor_b32 %3, %3, %8\n"         \
      "v_xor_b32 %4, %4, %8\n v_xor_b32 %5, %5, %8\n v_xor_b32 %6, %6, %8\n v_xor_b32 %7, %7, %8\n"         \
      "v_add_u32 %0, %0, %8\n v_add_u32 %1, %1, %8\n v_add_u32 %2, %2, %8\n v_add_u32 %3, %3, %8\n"         \
      "v_add_u32 %4, %4, %8\n v_add_u32 %5, %5, %8\n v_add_u32 %6, %6, %8\n v_add_u32 %7, %7, %8"            \
      : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)                       \
      : "v"(b))

__global__ __launch_bounds__(256) void k_valu_peak(uint32_t* __restrict__ out, uint32_t iters, uint32_t seed) {
  uint32_t a0 = threadIdx.x + seed, a1 = a0 * 3u, a2 = a0 * 5u, a3 = a0 * 7u;
  uint32_t a4 = a0 * 9u, a5 = a0 * 11u, a6 = a0 * 13u, a7 = a0 * 15u;
  const uint32_t b = seed ^ (blockIdx.x * 0x9e3779b9u) ^ threadIdx.x;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q) TCR_PROBE_ROUND;
  }
  out[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

}  // namespace

extern "C" int32_t tcrnet_valu_peak(tcrnet_ctx* ctx, double* lane_instr_per_s, double* seconds) {
  using namespace tcr;
  if (!ctx || !lane_instr_per_s) return set_error(TCRNET_EINVAL, "NULL argument");
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_error(e, "set device");
  int cus = 0;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device)) != hipSuccess)
    return hip_error(e, "device attribute");
  // 4 SIMDs per CU x 8 waves per SIMD, 4 waves per block
  const uint32_t grid = (uint32_t)std::max(cus, 1) * 8;
  DevBuf out;
  if ((e = out.ensure((size_t)grid * 256 * 4)) != hipSuccess) return hip_error(e, "probe buffer");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_error(e, "event");
  }
  const uint32_t iters = 20000;
  hipLaunchKernelGGL(k_valu_peak, dim3(grid), dim3(256), 0, ctx->stream, out.as<uint32_t>(), 200u, 1u);
  (void)hipEventRecord(e0, ctx->stream);
  hipLaunchKernelGGL(k_valu_peak, dim3(grid), dim3(256), 0, ctx->stream, out.as<uint32_t>(), iters, 2u);
  (void)hipEventRecord(e1, ctx->stream);
  float ms = 0.f;
  e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_error(e, "probe");
  const double lanes = (double)grid * 256.0;
  *lane_instr_per_s = lanes * (double)iters * kPerIter / (ms * 1e-3);
  if (seconds) *seconds = ms * 1e-3;
  return TCRNET_OK;
}
