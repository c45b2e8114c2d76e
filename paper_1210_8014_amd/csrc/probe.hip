// probe.hip -- issue-rate probe of single VALU instructions on gfx950 (a
// measurement aid, built beside the library as libamrprobe.so; it is not
// part of the rendering path).
//
// Each kernel runs a loop whose body issues one instruction (or one
// compare-and-select pair) of the kind under test 32 times per lane (4 rounds
// over 8 independent register chains, so that no instruction waits on the
// one before it and the loop's own three scalar instructions are amortised), with every wave slot of the
// chip filled (blocks of 256 threads, several rounds of 8 waves per SIMD on
// all compute units).  The host times each launch with HIP events; every
// wave also reads the core-cycle counter and the constant-rate counter
// around its loop, so the clock the chip actually ran at is known, and the
// rate is reported both per actual cycle and per cycle of the nominal
// 2.4 GHz.  The chip's published fp32 rate, 157.3 TFLOP/s = 2 flop x 64
// lanes x 512 x 2.4 GHz, is 512 wave64 VALU instructions per cycle, the peak
// the bench's VALU fractions are taken against.  Only registers are touched
// until the chains are stored once at the end (so that the compiler keeps
// the loop).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

namespace {

constexpr int kChains = 8;
constexpr int kRounds = 4;  // steps per chain and loop iteration

// The kinds under test: name and wave64 instructions per chain step (two for
// the compare-and-select pairs, the compiler's usual select idioms).
#define AMR_PROBE_KINDS(X)                                         \
  X(kAddU32, "v_add_u32", 1)                                       \
  X(kSubU32, "v_sub_u32", 1)                                       \
  X(kXor, "v_xor_b32", 1)                                          \
  X(kAnd, "v_and_b32", 1)                                          \
  X(kOr, "v_or_b32", 1)                                            \
  X(kMov, "v_mov_b32", 1)                                          \
  X(kAddF32, "v_add_f32", 1)                                       \
  X(kMulF32, "v_mul_f32", 1)                                       \
  X(kMaxF32, "v_max_f32", 1)                                       \
  X(kFmacF32, "v_fmac_f32", 1)                                     \
  X(kFmaF32, "v_fma_f32", 1)                                       \
  X(kLshl, "v_lshlrev_b32", 1)                                     \
  X(kLshr, "v_lshrrev_b32", 1)                                     \
  X(kAshr, "v_ashrrev_i32", 1)                                     \
  X(kMinI32, "v_min_i32", 1)                                       \
  X(kBitop3, "v_bitop3_b32", 1)                                    \
  X(kOr3, "v_or3_b32", 1)                                          \
  X(kBfi, "v_bfi_b32", 1)                                          \
  X(kAndOr, "v_and_or_b32", 1)                                     \
  X(kLshlOr, "v_lshl_or_b32", 1)                                   \
  X(kAdd3U32, "v_add3_u32", 1)                                     \
  X(kAddcCo, "v_addc_co_u32 (carry in from an SGPR pair)", 1)     \
  X(kMulU24, "v_mul_u32_u24", 1)                                   \
  X(kBfe, "v_bfe_u32", 1)                                          \
  X(kCvtF32I32, "v_cvt_f32_i32", 1)                                \
  X(kCvtF32U32, "v_cvt_f32_u32", 1)                                \
  X(kFfbl, "v_ffbl_b32", 1)                                        \
  X(kMulLo, "v_mul_lo_u32", 1)                                     \
  X(kMadI64, "v_mad_i64_i32", 1)                                   \
  X(kLshlAddU64, "v_lshl_add_u64", 1)                              \
  X(kCmpU32, "v_cmp_gt_u32 (to an SGPR pair)", 1)                  \
  X(kCmpI64, "v_cmp_gt_i64 (to an SGPR pair)", 1)                  \
  X(kCndmaskE64, "v_cndmask_b32_e64 (SGPR-pair mask)", 1)          \
  X(kCndmaskVcc, "v_cndmask_b32_e32 (VCC not written in the loop)", 1) \
  X(kCmpSelVcc, "v_cmp_gt_u32 to VCC + v_cndmask_b32_e32", 2)      \
  X(kCmpSelE64, "v_cmp_gt_u32 to an SGPR pair + v_cndmask_b32_e64", 2)

#define AMR_PROBE_ENUM(e, n, c) e,
enum Kind { AMR_PROBE_KINDS(AMR_PROBE_ENUM) kNumKinds };
#define AMR_PROBE_NAME(e, n, c) n,
const char* kNames[kNumKinds] = {AMR_PROBE_KINDS(AMR_PROBE_NAME)};
#define AMR_PROBE_COUNT(e, n, c) c,
const int kInstrs[kNumKinds] = {AMR_PROBE_KINDS(AMR_PROBE_COUNT)};

// Keeps a scalar result live without an instruction.
#define AMR_PROBE_USE_S(m) asm volatile("" ::"s"(m))

template <int K>
__global__ __launch_bounds__(256) void k_probe(uint32_t* out, uint64_t* clk, int iters, uint32_t seed) {
  uint32_t r[kChains];
  for (int c = 0; c < kChains; ++c) r[c] = seed + threadIdx.x * 7u + c * 13u;
  uint64_t q[kChains];  // 64-bit chains for the 64-bit kinds
  for (int c = 0; c < kChains; ++c) q[c] = ((uint64_t)r[c] << 20) | r[c];
  const uint32_t b = seed | 1u, b2 = seed * 3u + threadIdx.x;  // two further register operands
  const uint64_t b64 = ((uint64_t)b2 << 32) | b;
  const uint64_t smask = 0x5555555555555555ull ^ seed;  // a lane mask in scalar registers
  const uint64_t c0 = (uint64_t)clock64();
  const uint64_t w0 = (uint64_t)wall_clock64();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        uint32_t& x = r[c];
        const uint32_t y = r[(c + 1) % kChains];
        if constexpr (K == kAddU32) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kSubU32) asm volatile("v_sub_u32 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kXor) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kAnd) asm volatile("v_and_b32 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kOr) asm volatile("v_or_b32 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kMov) asm volatile("v_mov_b32 %0, %1" : "=v"(x) : "v"(y));
        if constexpr (K == kAddF32) asm volatile("v_add_f32 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kMulF32) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kMaxF32) asm volatile("v_max_f32 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kFmacF32) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(x) : "v"(b), "v"(b2));
        if constexpr (K == kFmaF32) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x) : "v"(b), "v"(b2));
        if constexpr (K == kLshl) asm volatile("v_lshlrev_b32 %0, %1, %0" : "+v"(x) : "v"(b));
        if constexpr (K == kLshr) asm volatile("v_lshrrev_b32 %0, %1, %0" : "+v"(x) : "v"(b));
        if constexpr (K == kAshr) asm volatile("v_ashrrev_i32 %0, %1, %0" : "+v"(x) : "v"(b));
        if constexpr (K == kMinI32) asm volatile("v_min_i32 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kBitop3) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(x) : "v"(b), "v"(b2));
        if constexpr (K == kOr3) asm volatile("v_or3_b32 %0, %0, %1, %2" : "+v"(x) : "v"(b), "v"(b2));
        if constexpr (K == kBfi) asm volatile("v_bfi_b32 %0, %1, %0, %2" : "+v"(x) : "v"(b), "v"(b2));
        if constexpr (K == kAndOr) asm volatile("v_and_or_b32 %0, %0, %1, %2" : "+v"(x) : "v"(b), "v"(b2));
        if constexpr (K == kLshlOr) asm volatile("v_lshl_or_b32 %0, %0, 3, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kAdd3U32) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(x) : "v"(b), "v"(b2));
        if constexpr (K == kAddcCo) {
          uint64_t carry;
          asm volatile("v_addc_co_u32 %0, %1, %0, %2, %3" : "+v"(x), "=s"(carry) : "v"(b), "s"(smask));
        }
        if constexpr (K == kMulU24) asm volatile("v_mul_u32_u24 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kBfe) asm volatile("v_bfe_u32 %0, %0, 3, 9" : "+v"(x));
        if constexpr (K == kCvtF32I32) asm volatile("v_cvt_f32_i32 %0, %0" : "+v"(x));
        if constexpr (K == kCvtF32U32) asm volatile("v_cvt_f32_u32 %0, %0" : "+v"(x));
        if constexpr (K == kFfbl) asm volatile("v_ffbl_b32 %0, %0" : "+v"(x));
        if constexpr (K == kMulLo) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x) : "v"(b));
        if constexpr (K == kMadI64) {
          uint64_t carry;
          asm volatile("v_mad_i64_i32 %0, %1, %2, %2, %0" : "+v"(q[c]), "=s"(carry) : "v"(b));
        }
        if constexpr (K == kLshlAddU64) asm volatile("v_lshl_add_u64 %0, %0, 1, %1" : "+v"(q[c]) : "v"(b64));
        if constexpr (K == kCmpU32) {
          uint64_t m;
          asm volatile("v_cmp_gt_u32 %0, %1, %2" : "=s"(m) : "v"(x), "v"(y));
          AMR_PROBE_USE_S(m);
        }
        if constexpr (K == kCmpI64) {
          uint64_t m;
          asm volatile("v_cmp_gt_i64 %0, %1, %2" : "=s"(m) : "v"(q[c]), "v"(q[(c + 1) % kChains]));
          AMR_PROBE_USE_S(m);
        }
        if constexpr (K == kCndmaskE64) asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(x) : "v"(b), "s"(smask));
        if constexpr (K == kCndmaskVcc) asm volatile("v_cndmask_b32_e32 %0, %0, %1, vcc" : "+v"(x) : "v"(b));
        if constexpr (K == kCmpSelVcc)
          asm volatile("v_cmp_gt_u32 vcc, %1, %2\n\tv_cndmask_b32_e32 %0, %0, %2, vcc" : "+v"(x) : "v"(y), "v"(b) : "vcc");
        if constexpr (K == kCmpSelE64) {
          uint64_t m;
          asm volatile("v_cmp_gt_u32 %1, %2, %3\n\tv_cndmask_b32_e64 %0, %0, %3, %1" : "+v"(x), "=&s"(m) : "v"(y), "v"(b));
        }
      }
    }
  }
  const uint64_t c1 = (uint64_t)clock64();
  const uint64_t w1 = (uint64_t)wall_clock64();
  uint32_t acc = 0;
  for (int c = 0; c < kChains; ++c) acc ^= r[c] ^ (uint32_t)q[c] ^ (uint32_t)(q[c] >> 32);
  out[blockIdx.x * 256 + threadIdx.x] = acc;
  if ((threadIdx.x & 63) == 0) {
    const uint32_t wave = blockIdx.x * 4 + threadIdx.x / 64;
    clk[2 * wave] = c1 - c0;
    clk[2 * wave + 1] = w1 - w0;
  }
}

template <int K>
hipError_t launch(uint32_t* out, uint64_t* clk, int blocks, int iters, hipStream_t s) {
  hipLaunchKernelGGL(k_probe<K>, dim3(blocks), dim3(256), 0, s, out, clk, iters, 12345u);
  return hipGetLastError();
}

hipError_t launch_kind(int k, uint32_t* out, uint64_t* clk, int blocks, int iters, hipStream_t s) {
#define AMR_PROBE_CASE(e, n, c) \
  case e:                       \
    return launch<e>(out, clk, blocks, iters, s);
  switch (k) { AMR_PROBE_KINDS(AMR_PROBE_CASE) }
  return hipErrorInvalidValue;
}

}  // namespace

extern "C" {

int32_t amrprobe_kinds(void) { return kNumKinds; }
const char* amrprobe_name(int32_t k) { return (k >= 0 && k < kNumKinds) ? kNames[k] : "invalid"; }
// wave64 instructions per lane and loop iteration of kind k (0 if no such kind)
int32_t amrprobe_per_iter(int32_t k) { return (k >= 0 && k < kNumKinds) ? kChains * kRounds * kInstrs[k] : 0; }

// Runs kind k once untimed and reps times timed on the current device:
// blocks x 256 threads, iters loop iterations of amrprobe_per_iter(k)
// instructions per lane.  ms[reps] receives each timed launch and mhz[reps]
// the core clock over it (core cycles over constant-rate ticks, summed over
// every wave of the launch, times the constant rate).  Returns 0 or a
// hipError_t.
int32_t amrprobe_run(int32_t k, int32_t blocks, int32_t iters, int32_t reps, float* ms, float* mhz) {
  if (k < 0 || k >= kNumKinds || blocks < 1 || blocks > (1 << 20) || iters < 1 || reps < 1 || !ms || !mhz)
    return (int32_t)hipErrorInvalidValue;
  int dev = 0, wall_khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return (int32_t)e;
  if (wall_khz <= 0) return (int32_t)hipErrorInvalidValue;
  const size_t waves = (size_t)blocks * 4;
  uint32_t* out = nullptr;
  uint64_t* clk = nullptr;
  uint64_t* host = (uint64_t*)malloc(waves * 2 * sizeof(uint64_t));
  if (!host) return (int32_t)hipErrorOutOfMemory;
  e = hipMalloc((void**)&out, (size_t)blocks * 256 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&clk, waves * 2 * sizeof(uint64_t));
  hipEvent_t a = nullptr, b = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = launch_kind(k, out, clk, blocks, iters, nullptr);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = hipEventRecord(a, nullptr);
    if (e == hipSuccess) e = launch_kind(k, out, clk, blocks, iters, nullptr);
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms[r], a, b);
    if (e == hipSuccess) e = hipMemcpy(host, clk, waves * 2 * sizeof(uint64_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
      double cycles = 0.0, ticks = 0.0;
      for (size_t w = 0; w < waves; ++w) {
        cycles += (double)host[2 * w];
        ticks += (double)host[2 * w + 1];
      }
      mhz[r] = ticks > 0.0 ? (float)(cycles / ticks * wall_khz * 1e-3) : 0.0f;
    }
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (out) (void)hipFree(out);
  if (clk) (void)hipFree(clk);
  free(host);
  return (int32_t)e;
}

}  // extern "C"
