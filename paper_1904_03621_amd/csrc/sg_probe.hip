// sg_probe.hip -- VALU issue-rate probe: the measured denominator of the
// enumeration kernel's roofline.  Each lane runs long chains of one VALU
// instruction kind over 8 independent accumulators (inline asm, so the
// compiler cannot fold or reorder them); the rate is lane-instructions per
// second over a grid that fills every SIMD.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sg {

constexpr int kProbeIters = 4096;
constexpr int kProbeThreads = 256;
constexpr int kProbeMixBase = 21;  // first instruction-mix code (after the single kinds)

// Instruction kinds measured (one asm template each; %0 accumulates, %1 and
// %2 are loop-invariant operands).
#define SG_PROBE_OPS(X)                                 \
  X(0, "v_add_f32 %0, %0, %1")                          \
  X(1, "v_min3_f32 %0, %0, %1, %2")                     \
  X(2, "v_add_u32 %0, %0, %1")                          \
  X(3, "v_min3_i32 %0, %0, %1, %2")                     \
  X(4, "v_fma_f32 %0, %0, %1, %2")                      \
  X(5, "v_min_f32 %0, %0, %1")                          \
  X(6, "v_or_b32 %0, %0, %1")                           \
  X(7, "v_or3_b32 %0, %0, %1, %2")                      \
  X(8, "v_add3_u32 %0, %0, %1, %2")                     \
  X(9, "v_max3_f32 %0, %0, %1, %2")                     \
  X(10, "v_min_i32 %0, %0, %1")                         \
  X(11, "v_sub_f32 %0, %1, %0")                         \
  X(12, "v_and_or_b32 %0, %0, %1, %2")                  \
  X(13, "v_med3_f32 %0, %0, %1, %2")                    \
  X(14, "v_pk_add_u16 %0, %0, %1")                      \
  X(15, "v_pk_min_i16 %0, %0, %1")                      \
  X(16, "v_exp_f32 %0, %1")                             \
  X(17, "v_sub_u32 %0, %1, %0")                         \
  X(18, "v_and_b32 %0, %0, %1")                         \
  X(19, "v_cvt_i32_f32 %0, %1")                         \
  X(20, "v_lshl_add_u32 %0, %0, 16, %1")

template <int kOp>
__global__ __launch_bounds__(kProbeThreads) void k_probe(uint32_t seed, uint32_t* out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a0 = t ^ seed, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5,
           a6 = a0 + 6, a7 = a0 + 7;
  // small positive float bit patterns keep the float chains finite
  a0 = 0x3f800000u | (a0 & 0xffu); a1 = 0x3f800000u | (a1 & 0xffu);
  a2 = 0x3f800000u | (a2 & 0xffu); a3 = 0x3f800000u | (a3 & 0xffu);
  a4 = 0x3f800000u | (a4 & 0xffu); a5 = 0x3f800000u | (a5 & 0xffu);
  a6 = 0x3f800000u | (a6 & 0xffu); a7 = 0x3f800000u | (a7 & 0xffu);
  const uint32_t b = 0x33800000u + (seed & 7u), c = 0x34400000u + (seed & 3u);
  for (int it = 0; it < kProbeIters; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (false) {}
#define ONE(code, str) \
      else if (kOp == code) { \
        asm volatile(str : "+v"(a0) : "v"(b), "v"(c)); asm volatile(str : "+v"(a1) : "v"(b), "v"(c)); \
        asm volatile(str : "+v"(a2) : "v"(b), "v"(c)); asm volatile(str : "+v"(a3) : "v"(b), "v"(c)); \
        asm volatile(str : "+v"(a4) : "v"(b), "v"(c)); asm volatile(str : "+v"(a5) : "v"(b), "v"(c)); \
        asm volatile(str : "+v"(a6) : "v"(b), "v"(c)); asm volatile(str : "+v"(a7) : "v"(b), "v"(c)); }
      SG_PROBE_OPS(ONE)
#undef ONE
    }
  }
  const uint32_t x = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
  if (x == 0x12345678u) out[0] = t;  // keeps the chains live
}

// Instruction mixes of the search walk's inner steps, 8 independent chains per
// lane, each asm block two Gray steps (two states):
//   kMix 0 (fp32 walk): ga = g + w0; g = ga + w1; m = min3(m, ga, g)
//          -- two adds and one 3-input min, 3 instructions per 2 states;
//   kMix 1 (two 16-bit fields per 32-bit word): g += p0; a &= g; g -= p1; a &= g
//          -- an integer add and an AND per step, 4 instructions per 2 states.
//   kMix 2: kMix 1 with one chain per lane (the walk's dependence: every add
//          waits for the last, every AND for the last AND and its add);
//   kMix 3: kMix 1 with two chains per lane;
//   kMix 4: kMix 0 with one chain per lane;
//   kMix 5: kMix 2 with 57 more registers live through the loop (the walk
//          kernel's register footprint: 64 VGPRs per lane at 8 waves/SIMD);
//   kMix 6: kMix 2 unrolled into one straight run of 1024 steps per loop
//          iteration (the walk kernel's long unrolled blocks).
constexpr int kMixInsts[7] = {3, 4, 4, 4, 3, 4, 4};

template <int kMix>
__global__ __launch_bounds__(kProbeThreads) void k_probe_mix(uint32_t seed, uint32_t* out) {
  constexpr int kChains = kMix == 2 || kMix == 4 || kMix >= 5 ? 1 : kMix == 3 ? 2 : 8;
  constexpr int kUnroll = kMix == 6 ? 16 : 1;  // asm blocks per chain and loop pass: x kUnroll
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t g[8], m[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    g[k] = 0x3f800000u | ((t + k) & 0xffu);
    m[k] = g[k];
  }
  const uint32_t w0 = 0x33800000u + (seed & 7u), w1 = 0xb3800000u + (seed & 3u);
  uint32_t x[57];
#pragma unroll
  for (int k = 0; k < 57; ++k) x[k] = t * (k + 3) + seed;
  for (int it = 0; it < kProbeIters / kUnroll; ++it) {
    if (kMix == 5) {
#pragma unroll
      for (int k = 0; k < 57; ++k) asm volatile("" : "+v"(x[k]));
    }
#pragma unroll
    for (int u = 0; u < 4 * 8 / kChains * kUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < kChains; ++k) {
        uint32_t ga;
        if (kMix == 0 || kMix == 4) {
          asm volatile(
              "v_add_f32 %1, %0, %3\n\t"
              "v_add_f32 %0, %1, %4\n\t"
              "v_min3_f32 %2, %2, %1, %0"
              : "+v"(g[k]), "=&v"(ga), "+v"(m[k])
              : "v"(w0), "v"(w1));
        } else {
          asm volatile(
              "v_add_u32 %0, %0, %2\n\t"
              "v_and_b32 %1, %1, %0\n\t"
              "v_sub_u32 %0, %0, %3\n\t"
              "v_and_b32 %1, %1, %0"
              : "+v"(g[k]), "+v"(m[k])
              : "v"(w0), "v"(w1));
        }
      }
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= g[k] ^ m[k];
  if (kMix == 5) {
#pragma unroll
    for (int k = 0; k < 57; ++k) r ^= x[k];
  }
  if (r == 0x12345678u) out[0] = t;  // keeps the chains live
}

// Lane-instructions per second of instruction kind `op` (SG_PROBE_OPS), over
// `waves_per_simd` resident waves per SIMD on every CU.  Returns < 0 on error.
double probe_valu(int op, int waves_per_simd) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1.0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return -1.0;
  const int blocks = prop.multiProcessorCount * 4 * waves_per_simd * 64 / kProbeThreads;
  uint32_t* out = nullptr;
  if (hipMalloc(&out, sizeof(uint32_t)) != hipSuccess) return -1.0;
  hipStream_t st;
  if (hipStreamCreate(&st) != hipSuccess) return -1.0;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  auto launch = [&](uint32_t seed) {
    switch (op) {
#define L(code, str)                                                                       \
  case code:                                                                              \
    hipLaunchKernelGGL(k_probe<code>, dim3(blocks), dim3(kProbeThreads), 0, st, seed, out); \
    break;
      SG_PROBE_OPS(L)
#undef L
      case kProbeMixBase:
        hipLaunchKernelGGL(k_probe_mix<0>, dim3(blocks), dim3(kProbeThreads), 0, st, seed, out);
        break;
      case kProbeMixBase + 1:
        hipLaunchKernelGGL(k_probe_mix<1>, dim3(blocks), dim3(kProbeThreads), 0, st, seed, out);
        break;
      case kProbeMixBase + 2:
        hipLaunchKernelGGL(k_probe_mix<2>, dim3(blocks), dim3(kProbeThreads), 0, st, seed, out);
        break;
      case kProbeMixBase + 3:
        hipLaunchKernelGGL(k_probe_mix<3>, dim3(blocks), dim3(kProbeThreads), 0, st, seed, out);
        break;
      case kProbeMixBase + 4:
        hipLaunchKernelGGL(k_probe_mix<4>, dim3(blocks), dim3(kProbeThreads), 0, st, seed, out);
        break;
      case kProbeMixBase + 5:
        hipLaunchKernelGGL(k_probe_mix<5>, dim3(blocks), dim3(kProbeThreads), 0, st, seed, out);
        break;
      case kProbeMixBase + 6:
        hipLaunchKernelGGL(k_probe_mix<6>, dim3(blocks), dim3(kProbeThreads), 0, st, seed, out);
        break;
      default: break;
    }
  };
  launch(1u);  // warm-up
  (void)hipEventRecord(a, st);
  for (int r = 0; r < 4; ++r) launch(2u + r);
  (void)hipEventRecord(b, st);
  double rate = -1.0;
  if (hipEventSynchronize(b) == hipSuccess) {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    const double per_asm = op >= kProbeMixBase ? kMixInsts[op - kProbeMixBase] : 1.0;
    const double lane_ops = 4.0 * (double)blocks * kProbeThreads * kProbeIters * 4 * 8 * per_asm;
    rate = ms > 0.0f ? lane_ops / (ms * 1e-3) : -1.0;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(st);
  (void)hipFree(out);
  return rate;
}

}  // namespace sg
