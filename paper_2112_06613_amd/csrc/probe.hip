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

// Issue rates of single instruction forms: the same eight chains a wave,
// each round one form only.  The forms are those the bit-vector step and its
// within-k tests compile to (and their alternatives), so the rates price the
// pair kernel's instruction mix: on gfx950 some 32-bit forms issue at twice
// the rate of others (see tcrnet_valu_rates).
#define TCR_CH8(INS)                                                                              \
  asm volatile(INS(0) INS(1) INS(2) INS(3) INS(4) INS(5) INS(6) INS(7)                            \
               : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)   \
               : "v"(b), "v"(c))
#define TCR_XOR(i) "v_xor_b32 %" #i ", %" #i ", %8\n"
#define TCR_ADD(i) "v_add_u32 %" #i ", %" #i ", %8\n"
#define TCR_AND(i) "v_and_b32 %" #i ", %" #i ", %8\n"
#define TCR_BITOP3(i) "v_bitop3_b32 %" #i ", %" #i ", %8, %9 bitop3:0xde\n"
#define TCR_PKADD(i) "v_pk_add_u16 %" #i ", %" #i ", %8\n"
#define TCR_ADD3(i) "v_add3_u32 %" #i ", %" #i ", %8, %9\n"
#define TCR_OR3(i) "v_or3_b32 %" #i ", %" #i ", %8, %9\n"
#define TCR_MIN(i) "v_min_u32 %" #i ", %" #i ", %8\n"
#define TCR_MINSDWA(i) \
  "v_min_u32_sdwa %" #i ", %" #i ", %8 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1\n"
#define TCR_LSHL(i) "v_lshlrev_b32 %" #i ", 1, %" #i "\n"
#define TCR_BCNT(i) "v_bcnt_u32_b32 %" #i ", %" #i ", %8\n"
#define TCR_FORM_KERNEL(NAME, INS)                                                                 \
  __global__ __launch_bounds__(256) void NAME(uint32_t* __restrict__ out, uint32_t iters, uint32_t seed) { \
    uint32_t a0 = threadIdx.x + seed, a1 = a0 * 3u, a2 = a0 * 5u, a3 = a0 * 7u;                    \
    uint32_t a4 = a0 * 9u, a5 = a0 * 11u, a6 = a0 * 13u, a7 = a0 * 15u;                            \
    const uint32_t b = seed ^ (blockIdx.x * 0x9e3779b9u) ^ threadIdx.x, c = b * 7u;               \
    for (uint32_t it = 0; it < iters; ++it) {                                                      \
      _Pragma("unroll") for (int q = 0; q < 8; ++q) TCR_CH8(INS);                                  \
    }                                                                                              \
    out[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;  \
  }
TCR_FORM_KERNEL(k_form_xor, TCR_XOR)
TCR_FORM_KERNEL(k_form_add, TCR_ADD)
TCR_FORM_KERNEL(k_form_and, TCR_AND)
TCR_FORM_KERNEL(k_form_bitop3, TCR_BITOP3)
TCR_FORM_KERNEL(k_form_pkadd, TCR_PKADD)
TCR_FORM_KERNEL(k_form_add3, TCR_ADD3)
TCR_FORM_KERNEL(k_form_or3, TCR_OR3)
TCR_FORM_KERNEL(k_form_min, TCR_MIN)
TCR_FORM_KERNEL(k_form_minsdwa, TCR_MINSDWA)
TCR_FORM_KERNEL(k_form_lshl, TCR_LSHL)
TCR_FORM_KERNEL(k_form_bcnt, TCR_BCNT)

// v_cmp into VCC (the compare that feeds every step's ballot): eight
// independent compares a round, the mask folded into a chain so none is dead
__global__ __launch_bounds__(256) void k_form_cmp(uint32_t* __restrict__ out, uint32_t iters, uint32_t seed) {
  const uint32_t a0 = threadIdx.x + seed, b = seed ^ threadIdx.x;
  uint32_t acc = 0;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      uint64_t m;
      asm volatile(
          "v_cmp_eq_u32 vcc, %1, %2\n v_cmp_eq_u32 vcc, %1, %2\n v_cmp_eq_u32 vcc, %1, %2\n"
          "v_cmp_eq_u32 vcc, %1, %2\n v_cmp_eq_u32 vcc, %1, %2\n v_cmp_eq_u32 vcc, %1, %2\n"
          "v_cmp_eq_u32 vcc, %1, %2\n v_cmp_eq_u32 vcc, %1, %2\n s_mov_b64 %0, vcc"
          : "=s"(m)
          : "v"(a0), "v"(b)
          : "vcc");
      acc ^= (uint32_t)m;
    }
  }
  out[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc ^ a0;
}

typedef void (*FormKernel)(uint32_t*, uint32_t, uint32_t);
struct Form {
  const char* name;
  FormKernel kernel;
};
const Form kForms[] = {
    {"v_xor_b32", k_form_xor},       {"v_add_u32", k_form_add},          {"v_and_b32", k_form_and},
    {"v_bitop3_b32", k_form_bitop3}, {"v_pk_add_u16", k_form_pkadd},     {"v_add3_u32", k_form_add3},
    {"v_or3_b32", k_form_or3},       {"v_min_u32", k_form_min},          {"v_min_u32_sdwa", k_form_minsdwa},
    {"v_lshlrev_b32", k_form_lshl},  {"v_bcnt_u32_b32", k_form_bcnt},    {"v_cmp_eq_u32", k_form_cmp},
};
constexpr uint32_t kNumForms = sizeof(kForms) / sizeof(kForms[0]);

}  // namespace

extern "C" const char* tcrnet_valu_form_name(uint32_t i) { return i < kNumForms ? kForms[i].name : nullptr; }

extern "C" int32_t tcrnet_valu_rates(tcrnet_ctx* ctx, double* lane_instr_per_s, uint32_t capacity,
                                     uint32_t* n_forms) {
  using namespace tcr;
  if (!ctx || !n_forms || (capacity && !lane_instr_per_s)) return set_error(TCRNET_EINVAL, "NULL argument");
  *n_forms = kNumForms;
  if (capacity < kNumForms) return set_error(TCRNET_EINVAL, "rates array holds %u of %u forms", capacity, kNumForms);
  hipError_t e;
  if ((e = hipSetDevice(ctx->device)) != hipSuccess) return hip_error(e, "set device");
  int cus = 0;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device)) != hipSuccess)
    return hip_error(e, "device attribute");
  const uint32_t grid = (uint32_t)std::max(cus, 1) * 8;  // 8 waves per SIMD
  DevBuf out;
  if ((e = out.ensure((size_t)grid * 256 * 4)) != hipSuccess) return hip_error(e, "probe buffer");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_error(e, "event");
  }
  const uint32_t iters = 2000;
  for (uint32_t f = 0; f < kNumForms && e == hipSuccess; ++f) {
    hipLaunchKernelGGL(kForms[f].kernel, dim3(grid), dim3(256), 0, ctx->stream, out.as<uint32_t>(), 100u, 1u);
    (void)hipEventRecord(e0, ctx->stream);
    hipLaunchKernelGGL(kForms[f].kernel, dim3(grid), dim3(256), 0, ctx->stream, out.as<uint32_t>(), iters, 2u);
    (void)hipEventRecord(e1, ctx->stream);
    float ms = 0.f;
    e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) lane_instr_per_s[f] = (double)grid * 256.0 * iters * 64.0 / (ms * 1e-3);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_error(e, "rate probe");
  return TCRNET_OK;
}

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
