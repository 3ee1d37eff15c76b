// sg_logz.hip -- exact log Z(beta) and its gradients by exhaustive enumeration
// (the Boltzmann weight at inverse temperature beta of Sec. 5.2, summed over
// all 2^N states of Eq. 1).
//
//   log Z(beta) = -beta E0 + log sum_s exp(-beta (E(s) - E0))
//   d log Z / d J_ij = beta <s_i s_j>,   d log Z / d h_i = beta <s_i>
//
// E0 is the ground energy found by the low-spectrum search, so every shifted
// weight is at most 1.  The walk is the same Gray-code walk as the search
// (prefix per lane, free spins 0..n-1, low blocks of 2^U steps) but keeps its
// energy chain in fp64: only the shifted energy x = E - E0 is rounded to fp32
// for the exponent (v_exp_f32, base 2).
//
// Forward (kMode 0): per lane, fp32 sums of the 64 weights of a block are
// added into fp64 per-beta totals; a wave reduction and one fp64 atomic per
// wave give the per-instance sums.
//
// Backward (kMode 1): the gradient of sum_b g_b log Z(beta_b) needs, for every
// pair and every spin, sum_s omega(s) s_i s_j and sum_s omega(s) s_i with the
// combined weight omega = sum_b (g_b beta_b / Z_b) exp(-beta_b (E - E0)).
// Inside a block the low spins take all 64 configurations, so the block
// contributes the order <= 2 Walsh coefficients of omega over those spins
// (total, 6 singles, 15 pairs); they are built hierarchically while the block
// is walked (halves of a group differ in one spin).  Prefix spins are constant
// per lane and high spins constant per block, so:
//   prefix-involving moments  <- per-lane fp64 totals (Omega, A_f, M_g) times
//                                prefix signs, reduced at the end of the lane;
//   free x free pairs         <- per-block wave sums of the 22 coefficients
//                                times high-spin signs, kept in accumulators
//                                distributed over the lanes of the wave.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_internal.h"

namespace sg {

constexpr int kLzHigh = kLzFree - kU;
constexpr int kNCoef = 22;   // 1 + 6 + 15 order <= 2 Walsh coefficients over U = 6

// ------------------------------------------------------------------ prep

template <int kMode>
__global__ void k_lz_prep(LzArgs a, const float* __restrict__ J, double* q64,
                          const float* energies, float* e0_out, const double* logz,
                          const double* grad) {
  const int b = blockIdx.x;
  const int N = a.N;
  const float* Jb = J + (size_t)b * N * N;
  const int tid = threadIdx.x;
  if (tid < 2 * kBlockSteps) {
    const int par = tid / kBlockSteps, i = tid % kBlockSteps;
    const uint32_t x = (uint32_t)(i ^ (i >> 1)) ^ ((uint32_t)par << (kU - 1));
    double q = 0.0;
    for (int f = 0; f < kU; ++f)
      for (int g = f + 1; g < kU; ++g) {
        const double sf = ((x >> f) & 1u) ? 1.0 : -1.0, sg = ((x >> g) & 1u) ? 1.0 : -1.0;
        q -= (double)Jb[f * N + g] * sf * sg;
      }
    q64[(size_t)b * 2 * kBlockSteps + tid] = q;
  }
  double* acc = a.acc + (size_t)b * a.acc_stride;
  for (int k = tid; k < a.acc_stride; k += blockDim.x) acc[k] = 0.0;
  if (tid == 0) {
    for (int k = 0; k < a.nb; ++k) {
      const float bk = a.beta[k];
      if (!(bk > 0.0f) || !isfinite(bk)) atomicOr(a.sticky, kErrInval);
    }
    if (kMode == 0) {
      e0_out[b] = energies[(size_t)b * a.S];
    } else {
      for (int k = 0; k < kMaxBeta; ++k) {
        double c = 0.0;
        if (k < a.nb) {
          const double bk = (double)a.beta[k];
          // Z~_b = sum exp(-beta (E - E0)) = exp(log Z + beta E0)
          const double zt = exp(logz[(size_t)b * a.nb + k] + bk * (double)a.e0[b]);
          c = grad[(size_t)b * a.nb + k] * bk / zt;
        }
        a.coef[(size_t)b * kMaxBeta + k] = c;
      }
    }
  }
}

// ------------------------------------------------------- block Walsh walk
// Order <= 2 Walsh coefficients of the block weights over the low spins
// 0..K-1 of a group of 2^K consecutive steps.  Pairs (f < g) are stored at
// g (g - 1) / 2 + f, so a pair keeps its slot as K grows.

struct Coefs {
  float o;
  float s[kU];
  float p[kU * (kU - 1) / 2];
};

constexpr int pidx(int f, int g) { return g * (g - 1) / 2 + f; }

struct BlockWalk {
  double& D;             // chain: G - E0 of the current state (fp64)
  const double* W;       // [U] low fields of this block, sign of U-1 folded in
  const double* q;       // [64] low-low energies of this block's parity
  const float* c;        // [kMaxBeta] -beta / ln 2
  const float* w;        // [kMaxBeta] combined weights a_b
  int nb;
  float sgn5;            // value of spin U-1 in the block's first half

  __device__ inline float weight(float x) const {
    float om = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxBeta; ++k)
      if (k < nb) om = fmaf(w[k], __builtin_amdgcn_exp2f(c[k] * x), om);
    return om;
  }

  // state I of the block: step the chain to it (I > 0), return its weight
  template <int I>
  __device__ inline float step() {
    if (I > 0) {
      constexpr int f = __builtin_ctz(I > 0 ? I : 1);
      if (f == kU - 1) D = D + W[f];
      else if ((I >> (f + 1)) & 1) D = D + W[f];
      else D = D - W[f];
    }
    return weight((float)(D + q[I]));
  }

  template <int K, int I0>
  __device__ inline Coefs walk() {
    Coefs r;
    if constexpr (K == 0) {
      r.o = step<I0>();
    } else {
      const Coefs a = walk<K - 1, I0>();
      const Coefs b = walk<K - 1, I0 + (1 << (K - 1))>();
      // spin K-1 is constant on each half and opposite between them; its value
      // on the first half is bit K-1 of the low configuration gray(I0)
      constexpr int g = K - 1;
      constexpr bool up = ((I0 ^ (I0 >> 1)) >> g) & 1;
      r.o = a.o + b.o;
#pragma unroll
      for (int f = 0; f < g; ++f) r.s[f] = a.s[f] + b.s[f];
#pragma unroll
      for (int f1 = 1; f1 < g; ++f1)
#pragma unroll
        for (int f0 = 0; f0 < f1; ++f0) r.p[pidx(f0, f1)] = a.p[pidx(f0, f1)] + b.p[pidx(f0, f1)];
      if (g == kU - 1) {
        r.s[g] = sgn5 * (a.o - b.o);
#pragma unroll
        for (int f = 0; f < g; ++f) r.p[pidx(f, g)] = sgn5 * (a.s[f] - b.s[f]);
      } else {
        r.s[g] = up ? a.o - b.o : b.o - a.o;
#pragma unroll
        for (int f = 0; f < g; ++f) r.p[pidx(f, g)] = up ? a.s[f] - b.s[f] : b.s[f] - a.s[f];
      }
    }
    return r;
  }
};

// wave sum of a double (every lane gets the total)
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Free x free pair slots distributed over the 64 lanes of a wave: slot s is
// a low-low pair (s < 15), a low-high pair, or a high-high pair; `coef` is the
// block coefficient it sums, `mask` the high spins whose signs multiply it.
__device__ inline void lz_slot(int s, int H, int N, int* coef, uint32_t* mask, int* target) {
  if (s < 15) {
    int g = 1;
    while (pidx(0, g + 1) <= s) ++g;
    const int f = s - pidx(0, g);
    *coef = 1 + kU + s;
    *mask = 0;
    *target = f * N + g;
    return;
  }
  s -= 15;
  if (s < kU * H) {
    const int f = s % kU, k = s / kU;
    *coef = 1 + f;
    *mask = 1u << k;
    *target = f * N + (kU + k);
    return;
  }
  s -= kU * H;
  int k1 = 1;
  while (pidx(0, k1 + 1) <= s) ++k1;
  const int k0 = s - pidx(0, k1);
  *coef = 0;
  *mask = (1u << k0) | (1u << k1);
  *target = (kU + k0) * N + (kU + k1);
}

// ------------------------------------------------------------------ walk

template <int kMode>
__global__ __launch_bounds__(256) void k_logz(LzArgs a, const float* __restrict__ J,
                                              const float* __restrict__ h,
                                              const double* __restrict__ table64,
                                              const double* __restrict__ q64, int bpi) {
  constexpr int U = kU;
  __shared__ double s_y[kLzHigh * 256];
  __shared__ float s_c[kMode ? 4 * kNCoef * 64 : 1];
  __shared__ float s_t[kMode ? 4 * kNCoef : 1];

  const int b = blockIdx.x / bpi;
  const int blk = blockIdx.x - b * bpi;
  const int tid = threadIdx.x;
  const int N = a.N, n = a.n, H = n - U;
  const int64_t lane = (int64_t)blk * 256 + tid;
  const bool valid = lane < a.lanes;
  const uint64_t p = valid ? (uint64_t)lane : 0ull;
  const float* Jt = J + (size_t)b * N * N;
  const float* ht = h + (size_t)b * N;
  const double* tab = table64 + ((size_t)b * a.table_recs + (size_t)a.table_offset) * 8;

  // ---- per-lane init (fp64)
  double WL[U];
  double ysum = 0.0;
#pragma unroll
  for (int f = 0; f < U; ++f) {
    double acc = 0.0;
    for (int q = n; q < N; ++q) {
      const double jq = (double)Jt[f * N + q];
      acc += ((p >> (q - n)) & 1ull) ? jq : -jq;
    }
    ysum += acc;
    WL[f] = 2.0 * acc;
  }
  for (int f = U; f < n; ++f) {
    double acc = 0.0;
    for (int q = n; q < N; ++q) {
      const double jq = (double)Jt[f * N + q];
      acc += ((p >> (q - n)) & 1ull) ? jq : -jq;
    }
    ysum += acc;
    s_y[(f - U) * 256 + tid] = 2.0 * acc;
  }
  double EP = 0.0;
  for (int q = n; q < N; ++q) {
    const double sq = ((p >> (q - n)) & 1ull) ? 1.0 : -1.0;
    double f = (double)ht[q];
    for (int r = q + 1; r < N; ++r) {
      const double jr = (double)Jt[q * N + r];
      f += ((p >> (r - n)) & 1ull) ? jr : -jr;
    }
    EP -= sq * f;
  }
  // invalid lanes: a huge shifted energy makes every weight 0
  double D = valid ? EP + ysum + tab[1] - (double)a.e0[b] : 1e30;

  float cb[kMaxBeta], wb[kMaxBeta];
#pragma unroll
  for (int k = 0; k < kMaxBeta; ++k) {
    const bool on = k < a.nb;
    cb[k] = on ? -a.beta[k] * 1.4426950408889634f : 0.0f;
    wb[k] = kMode == 0 ? 1.0f : (on ? (float)a.coef[(size_t)b * kMaxBeta + k] : 0.0f);
  }
  const double* qb0 = q64 + (size_t)b * 2 * kBlockSteps;

  // per-lane totals
  double L[kMaxBeta] = {0.0, 0.0, 0.0, 0.0};  // forward
  double Om = 0.0, A[U], M[kLzHigh];            // backward
#pragma unroll
  for (int f = 0; f < U; ++f) A[f] = 0.0;
#pragma unroll
  for (int k = 0; k < kLzHigh; ++k) M[k] = 0.0;
  // distributed free x free slots of this lane
  const int ln = tid & 63, wv = tid >> 6;
  const int nslots = 15 + U * H + H * (H - 1) / 2;
  int sc[2] = {0, 0}, st[2] = {0, 0};
  uint32_t sm[2] = {0u, 0u};
  double dacc[2] = {0.0, 0.0};
  if (kMode == 1) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
      if (ln + 64 * r < nslots) lz_slot(ln + 64 * r, H, N, &sc[r], &sm[r], &st[r]);
  }
  __syncthreads();  // s_y

  const uint32_t nblocks = 1u << (n - U);
  for (uint32_t T = 0; T < nblocks; ++T) {
    const double* rec = tab + (size_t)T * 8;
    if (T != 0) {
      const int c = __builtin_ctz(T);
      const bool up = (T >> (c + 1)) & 1u;
      const double y = s_y[c * 256 + tid];
      D = up ? D + y : D - y;
      D = D + rec[0];
    }
    double W[U];
#pragma unroll
    for (int f = 0; f < U - 1; ++f) W[f] = WL[f] + rec[2 + f];
    W[U - 1] = ((T & 1u) ? WL[U - 1] : -WL[U - 1]) + rec[2 + U - 1];
    const double* qb = qb0 + (T & 1u) * kBlockSteps;

    if (kMode == 0) {
      float sb[kMaxBeta] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int i = 0; i < kBlockSteps; ++i) {
        if (i > 0) {
          const int f = __builtin_ctz(i);
          if (f == U - 1) D = D + W[f];
          else D = ((i >> (f + 1)) & 1) ? D + W[f] : D - W[f];
        }
        const float x = (float)(D + qb[i]);
#pragma unroll
        for (int k = 0; k < kMaxBeta; ++k)
          if (k < a.nb) sb[k] += __builtin_amdgcn_exp2f(cb[k] * x);
      }
#pragma unroll
      for (int k = 0; k < kMaxBeta; ++k) L[k] += (double)sb[k];
    } else {
      BlockWalk bw{D, W, qb, cb, wb, a.nb, (T & 1u) ? 1.0f : -1.0f};
      const Coefs C = bw.walk<U, 0>();
      // per-lane totals for the prefix-involving moments
      const uint32_t xh = T ^ (T >> 1);  // high spins of this block
      Om += (double)C.o;
#pragma unroll
      for (int f = 0; f < U; ++f) A[f] += (double)C.s[f];
#pragma unroll
      for (int k = 0; k < kLzHigh; ++k)
        if (k < H) M[k] += ((xh >> k) & 1u) ? (double)C.o : -(double)C.o;
      // wave sums of the 22 coefficients (transpose through LDS)
      float* cw = s_c + wv * kNCoef * 64;
      cw[0 * 64 + ln] = C.o;
#pragma unroll
      for (int f = 0; f < U; ++f) cw[(1 + f) * 64 + ln] = C.s[f];
#pragma unroll
      for (int k = 0; k < 15; ++k) cw[(1 + U + k) * 64 + ln] = C.p[k];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (ln < kNCoef) {
        float t0 = 0.0f, t1 = 0.0f, t2 = 0.0f, t3 = 0.0f;
        const float* row = cw + ln * 64;
#pragma unroll
        for (int j = 0; j < 64; j += 4) {
          t0 += row[j]; t1 += row[j + 1]; t2 += row[j + 2]; t3 += row[j + 3];
        }
        s_t[wv * kNCoef + ln] = (t0 + t1) + (t2 + t3);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        if (ln + 64 * r < nslots) {
          const float v = s_t[wv * kNCoef + sc[r]];
          // product of the high signs in the mask: -1 per high spin that is down
          const int downs = __popc(sm[r]) - __popc(sm[r] & xh);
          dacc[r] += (downs & 1) ? -(double)v : (double)v;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  }

  // ---- lane end: reduce over the lanes of the wave, one atomic per value
  double* acc = a.acc + (size_t)b * a.acc_stride;
  const bool lead = ln == 0;
  if (kMode == 0) {
#pragma unroll
    for (int k = 0; k < kMaxBeta; ++k) {
      if (k < a.nb) {
        const double t = wave_sum(L[k]);
        if (lead) atomicAdd(acc + k, t);
      }
    }
    return;
  }
  // prefix spins n .. N-1 are fixed per lane
  auto sp = [&](int q) -> double { return ((p >> (q - n)) & 1ull) ? 1.0 : -1.0; };
  // singles of the free spins
#pragma unroll
  for (int f = 0; f < U; ++f) {
    const double t = wave_sum(A[f]);
    if (lead) atomicAdd(acc + N * N + f, t);
  }
#pragma unroll
  for (int g = 0; g < kLzHigh; ++g) {
    if (g < H) {
      const double t = wave_sum(M[g]);
      if (lead) atomicAdd(acc + N * N + U + g, t);
    }
  }
  // prefix singles, prefix pairs, free x prefix pairs
  for (int q = n; q < N; ++q) {
    const double sq = sp(q);
    double t = wave_sum(sq * Om);
    if (lead) atomicAdd(acc + N * N + q, t);
    for (int r = q + 1; r < N; ++r) {
      t = wave_sum(sq * sp(r) * Om);
      if (lead) atomicAdd(acc + q * N + r, t);
    }
#pragma unroll
    for (int f = 0; f < U; ++f) {
      t = wave_sum(sq * A[f]);
      if (lead) atomicAdd(acc + f * N + q, t);
    }
#pragma unroll
    for (int g = 0; g < kLzHigh; ++g) {
      if (g < H) {
        t = wave_sum(sq * M[g]);
        if (lead) atomicAdd(acc + (U + g) * N + q, t);
      }
    }
  }
  // free x free pairs from the distributed slots
#pragma unroll
  for (int r = 0; r < 2; ++r)
    if (ln + 64 * r < nslots) atomicAdd(acc + st[r], dacc[r]);
}

// ---------------------------------------------------------------- finalize

__global__ void k_lz_final_fwd(LzArgs a, double* logz) {
  const int b = blockIdx.x;
  const int k = threadIdx.x;
  if (k < a.nb) {
    const double bk = (double)a.beta[k];
    logz[(size_t)b * a.nb + k] = -bk * (double)a.e0[b] + log(a.acc[(size_t)b * a.acc_stride + k]);
  }
}

__global__ void k_lz_final_bwd(LzArgs a, float* grad_J, float* grad_h) {
  const int b = blockIdx.y;
  const int N = a.N;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const double* acc = a.acc + (size_t)b * a.acc_stride;
  if (idx < N * N) {
    const int i = idx / N, j = idx % N;
    grad_J[(size_t)b * N * N + idx] = i < j ? (float)acc[idx] : 0.0f;
  } else if (idx < N * N + N) {
    grad_h[(size_t)b * N + (idx - N * N)] = (float)acc[idx];
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_lz_prep(int mode, const LzArgs& a, const float* J, double* q64,
                          const float* energies, float* e0_out, const double* logz,
                          const double* grad, hipStream_t st) {
  if (mode == 0)
    hipLaunchKernelGGL(k_lz_prep<0>, dim3(a.B), dim3(256), 0, st, a, J, q64, energies, e0_out,
                       logz, grad);
  else
    hipLaunchKernelGGL(k_lz_prep<1>, dim3(a.B), dim3(256), 0, st, a, J, q64, energies, e0_out,
                       logz, grad);
  return hipGetLastError();
}

hipError_t launch_logz(int mode, const LzArgs& a, const float* J, const float* h,
                       const double* table64, const double* q64, hipStream_t st) {
  const int bpi = (int)((a.lanes + 255) / 256);
  const dim3 grid((unsigned)((int64_t)bpi * a.B));
  if (mode == 0)
    hipLaunchKernelGGL(k_logz<0>, grid, dim3(256), 0, st, a, J, h, table64, q64, bpi);
  else
    hipLaunchKernelGGL(k_logz<1>, grid, dim3(256), 0, st, a, J, h, table64, q64, bpi);
  return hipGetLastError();
}

hipError_t launch_lz_final(int mode, const LzArgs& a, double* logz, float* grad_J, float* grad_h,
                           hipStream_t st) {
  if (mode == 0) {
    hipLaunchKernelGGL(k_lz_final_fwd, dim3(a.B), dim3(64), 0, st, a, logz);
  } else {
    const int tot = a.N * a.N + a.N;
    hipLaunchKernelGGL(k_lz_final_bwd, dim3((tot + 255) / 256, a.B), dim3(256), 0, st, a, grad_J,
                       grad_h);
  }
  return hipGetLastError();
}

}  // namespace sg
