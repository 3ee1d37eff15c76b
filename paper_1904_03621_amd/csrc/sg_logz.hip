// sg_logz.hip -- exact log Z(beta) and its gradients by exhaustive enumeration
// (the Boltzmann weight at inverse temperature beta of Sec. 5.2, summed over
// all 2^N states of Eq. 1).
//
//   log Z(beta) = -beta E0 + log sum_s exp(-beta (E(s) - E0))
//   d log Z / d J_ij = beta <s_i s_j>,   d log Z / d h_i = beta <s_i>
//
// E0 is the ground energy found by the low-spectrum search.  The walk uses the
// decomposition of the search (prefix per lane, free spins 0..n-1, blocks of
// the 2^U configurations of the U low spins with the high spins fixed), but it
// does not step through a block: inside block T the energy is
//   E(x) = K_T + sum_{f<U} phi_f s_f + Q(x),
// linear in the low spins apart from their own couplings Q, so
//   exp(-beta (E(x) - E0)) = P_T * prod_f c_f(s_f) * bq(x)
// with P_T = exp(-beta (K_T - sum|phi_f| + min Q - E0)), c_f = 1 for the sign
// that lowers phi_f s_f and exp(-2 beta |phi_f|) for the other, and
// bq(x) = exp(-beta (Q(x) - min Q)) a per-instance table.  Every factor except
// P_T lies in (0, 1], so nothing overflows; P_T is formed in fp64 range.
// K_T and phi_f are formed per block in fp64 from the lane's prefix fields,
// the block record and the field energy of the high spins (one fp64 update
// per block, at most 2^H - 1 terms).
//
// Forward (kMode 0): the 2^U weights of a block are a 2^(U/2) x 2^(U/2)
// contraction of the factor products of the lower and upper U/2 low spins
// with bq (U = 10 when N >= 10 and at most three beta: 32 x 32; U = 8 when
// N >= 8: 16 x 16; else U = 6: 8 x 8); block sums are fp32 (two chains of at
// most 32 fused multiply-adds over terms in (0, 1]: relative error at most
// 64 2^-24), lane totals fp64, one fp64 atomic per wave and beta.
//
// Backward: the gradient of sum_b g_b log Z(beta_b) needs, for every
// pair and every spin, sum_s omega(s) s_i s_j and sum_s omega(s) s_i with the
// combined weight omega = sum_b (g_b beta_b / Z_b) exp(-beta_b (E - E0)).
// omega is formed for each of the 64 states of a block of 6 low spins from the
// factors, and the block contributes the order <= 2 Walsh coefficients of
// omega over those spins (total, 6 singles, 15 pairs), built hierarchically
// over the Gray order of the block (the halves of a group differ in one
// spin).  When N >= 8 (k_lz_grad8) the blocks of 6 are the four sub-blocks
// of a record of 8 low spins, whose bound and factors are formed once per
// record; with N = 7, blocks of 6 (k_logz<1>).  Prefix spins
// are constant per lane and high spins constant per block, so:
//   prefix-involving moments  <- per-lane fp64 totals (Omega, A_f, M_g) times
//                                prefix signs, reduced at the end of the lane;
//   free x free pairs         <- per-block wave sums of the 22 coefficients
//                                times high-spin signs, kept in accumulators
//                                distributed over the lanes of the wave.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>

#include "sg_internal.h"

namespace sg {

constexpr int kLzHigh = kLzFree - kLzU;
constexpr int kNCoef = 22;   // 1 + 6 + 15 order <= 2 Walsh coefficients over U = 6
constexpr int kCoefStride = 24;  // a row's coefficient sums in LDS (16-byte rows)

// ------------------------------------------------------------------ prep
// One workgroup per instance: the low-low energies Q(x), their minimum, the
// bq tables of every beta, the accumulators cleared, E0 (forward) or the
// combined gradient weights g_b beta_b / Z~_b (backward).

// bq floats per beta: the forward reads bq by configuration (2^U entries);
// the gradient walk over blocks of 6 by configuration and by Gray step for
// both block parities (3 x 64), and over records of 8 by sub-block and Gray
// step (4 x 64).
template <int kMode, int U>
constexpr int lz_q_floats() {
  return kMode == 0 ? (1 << U) : (U == kLzUF ? (1 << U) : 3 * (1 << U));
}

// Low configuration (bit f: spin f up) of entry r of a bq table.
template <int kMode, int U>
__device__ inline int lz_q_config(int r) {
  constexpr int kSteps = 1 << U;
  if (kMode == 0) return r;
  if (U == kLzUF) {  // sub-block j: spins 6 and 7 = gray2(j), spins 0..5 = gray6(i)
    const int j = r >> kLzU, i = r & (kLzSteps - 1);
    return (i ^ (i >> 1)) | ((j ^ (j >> 1)) << kLzU);
  }
  if (r < kSteps) return r;
  const int i = r & (kSteps - 1);
  return (i ^ (i >> 1)) ^ ((r >= 2 * kSteps) ? (1 << (U - 1)) : 0);
}

template <int kMode, int U>
__global__ void k_lz_prep(LzArgs a, const float* __restrict__ J, float* lzq, double* lzqmin,
                          const float* energies, float* e0_out, const double* logz,
                          const double* grad) {
  constexpr int kSteps = 1 << U;
  constexpr int kQ = lz_q_floats<kMode, U>();
  static_assert(kQ <= lz_q_stride(U), "bq tables exceed their stride");
  __shared__ double s_q[kSteps];
  __shared__ double s_qmin;
  const int b = blockIdx.x;
  const int N = a.N;
  const float* Jb = J + (size_t)b * N * N;
  const int tid = threadIdx.x;
  for (int x = tid; x < kSteps; x += blockDim.x) {
    double q = 0.0;
    for (int f = 0; f < U; ++f)
      for (int g = f + 1; g < U; ++g) {
        const double sf = ((x >> f) & 1) ? 1.0 : -1.0, sg = ((x >> g) & 1) ? 1.0 : -1.0;
        q -= (double)Jb[f * N + g] * sf * sg;
      }
    s_q[x] = q;
  }
  __syncthreads();
  if (tid == 0) {
    double m = s_q[0];
    for (int x = 1; x < kSteps; ++x) m = fmin(m, s_q[x]);
    s_qmin = m;
    lzqmin[b] = m;
  }
  __syncthreads();
  const double qmin = s_qmin;
  for (int e = tid; e < a.nb * kQ; e += blockDim.x) {
    const int k = e / kQ, r = e - k * kQ;
    const int x = lz_q_config<kMode, U>(r);
    const double bk = (double)a.beta[k];
    lzq[((size_t)b * kMaxBeta + k) * lz_q_stride(U) + r] = (float)exp(-bk * (s_q[x] - qmin));
  }
  double* acc = a.acc + (size_t)b * a.acc_stride;
  for (int k = tid; k < a.acc_stride; k += blockDim.x) acc[k] = 0.0;
  // non-finite couplings or fields (the forward's search reports them too)
  bool bad = false;
  for (int k = tid; k < N * N + N; k += blockDim.x) {
    const float v = k < N * N ? Jb[k] : a.h_in[(size_t)b * N + (k - N * N)];
    if (k >= N * N || (k / N) < (k % N)) bad = bad || !isfinite(v);
  }
  if (bad) atomicOr(a.sticky, kErrNonFinite);
  if (tid == 0) {
    for (int k = 0; k < a.nb; ++k) {
      const float bk = a.beta[k];
      if (!(bk > 0.0f) || !isfinite(bk)) atomicOr(a.sticky, kErrInval);
    }
    if (kMode == 0) {
      e0_out[b] = energies[(size_t)b * a.S];
    } else {
      for (int k = 0; k < kMaxBeta; ++k) {
        double c = 0.0, c2 = 0.0;
        if (k < a.nb) {
          const double bk = (double)a.beta[k];
          // Z~_b = sum exp(-beta (E - E0)) = exp(log Z + beta E0)
          const double zt = exp(logz[(size_t)b * a.nb + k] + bk * (double)a.e0[b]);
          c = grad[(size_t)b * a.nb + k] * bk / zt;
          c2 = -bk * 1.4426950408889634;
        }
        a.coef[(size_t)b * 2 * kMaxBeta + k] = c;
        a.coef[(size_t)b * 2 * kMaxBeta + kMaxBeta + k] = c2;
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
  float s[kLzU];
  float p[kLzU * (kLzU - 1) / 2];
};

constexpr int pidx(int f, int g) { return g * (g - 1) / 2 + f; }

// kSub: a sub-block of a record of 8 (spin 5 starts down, B scaled by d);
// otherwise a block of 6 of either parity (spin 5's value on the first half
// in sgn5).
template <int NB, bool kSub>
struct BlockWalk {
  const float (*A)[8];   // [NB][8] factor products of spins 0-2, times the beta's weight
  const float (*B)[8];   // [NB][8] factor products of spins 3-5, indexed by the Gray
                         // code's bits (block parity folded in)
  const float* const* bq;  // [NB] -> bq by Gray step for this block (sub-block)
  const float* d;        // [NB] sub-block factors of spins 6 and 7 (kSub)
  float sgn5;            // value of spin U-1 in the block's first half (!kSub)

  // combined weight of Gray step I of the block
  template <int I>
  __device__ inline float step() const {
    constexpr int g = I ^ (I >> 1);
    float om = 0.0f;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      float bk = B[k][g >> 3];
      if constexpr (kSub) bk *= d[k];
      const float t = A[k][g & 7] * bk;
      om = k == 0 ? t * bq[k][I] : fmaf(t, bq[k][I], om);
    }
    return om;
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
      if (!kSub && g == kLzU - 1) {
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

// sum over the 16 lanes of a row (DPP row shifts; the row's last lane gets
// the total, the others partial sums)
__device__ inline float row_total(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, true));
  return v;
}

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
    *coef = 1 + kLzU + s;
    *mask = 0;
    *target = f * N + g;
    return;
  }
  s -= 15;
  if (s < kLzU * H) {
    const int f = s % kLzU, k = s / kLzU;
    *coef = 1 + f;
    *mask = 1u << k;
    *target = f * N + (kLzU + k);
    return;
  }
  s -= kLzU * H;
  int k1 = 1;
  while (pidx(0, k1 + 1) <= s) ++k1;
  const int k0 = s - pidx(0, k1);
  *coef = 0;
  *mask = (1u << k0) | (1u << k1);
  *target = (kLzU + k0) * N + (kLzU + k1);
}

// ------------------------------------------------------------------ walk

// Factor products of M spins: out[x] = prod_{j<M} (bit j of x ? cp[j] : cm[j]),
// x < 2^M, built one spin at a time (2^(j+1) products for spin j).
template <int M>
__device__ inline void factor_products(const float* cp, const float* cm, float* out) {
  out[0] = cm[0];
  out[1] = cp[0];
#pragma unroll
  for (int j = 1; j < M; ++j) {
#pragma unroll
    for (int x = 0; x < (1 << j); ++x) {
      out[x + (1 << j)] = out[x] * cp[j];
      out[x] = out[x] * cm[j];
    }
  }
}

// 2^x for any finite x in fp64 range: 2^n (n integer) times 2^f, f in [0, 1).
__device__ inline double exp2_wide(double x) {
  const double n = floor(x);
  const float f = (float)(x - n);
  const int ni = (int)fmin(fmax(n, -2000.0), 2000.0);
  return ldexp((double)__builtin_amdgcn_exp2f(f), ni);
}

// Workgroups per CU to fit: the backward for up to three beta keeps 3 waves
// per SIMD (at most 168 VGPRs; no scratch since the slot targets are formed
// again at the lane's end), 28% faster than 2 waves; with four beta it keeps
// 2.  The forward fits 4
// or more waves either way (5 measured no faster than 4).
template <int kMode, int NB>
constexpr int lz_min_blocks() {
  return kMode == 1 && NB == 4 ? 2 : 3;
}

// U low spins per block: kLzU for the gradient walk, kLzU or kLzUF for the
// partition sums (a block's 2^U weights are then a 2^(U/2) x 2^(U/2)
// contraction).
template <int kMode, int NB, int U>
__global__ __launch_bounds__(256, (lz_min_blocks<kMode, NB>())) void k_logz(LzArgs a, const float* __restrict__ J,
                                              const float* __restrict__ h,
                                              const double* __restrict__ table64,
                                              const float* __restrict__ lzq,
                                              const double* __restrict__ lzqmin, int bpi) {
  static_assert(kMode == 0 || U == kLzU, "the gradient walk takes blocks of kLzU spins");
  static_assert(U % 2 == 0 && U <= kLzFree, "blocks split into two equal halves");
  constexpr int kSteps = 1 << U;
  constexpr int kQ = kMode == 0 ? kSteps : 3 * kSteps;  // bq floats per beta
  constexpr int kHigh = kLzFree - U;
  constexpr int kM = 1 << (U / 2);
  __shared__ double s_y[kHigh * 256];
  __shared__ __align__(16) float s_c[kMode ? 4 * 4 * kCoefStride : 1];
  __shared__ float s_t[kMode ? 4 * kNCoef : 1];
  // bq tables in LDS: the gradient walk's, and the partition sums' of blocks
  // of 10 (12 KB for three beta: more than the scalar cache keeps between
  // blocks; blocks of 8 read their 3 KB with scalar loads)
  constexpr bool kBqLds = kMode == 1 || U > kLzUF;
  __shared__ float s_bq[kBqLds ? NB * kQ : 1];
  // the partition sums over records of 10 walk their blocks in pairs (below)
  // and keep the lane's fields of the low spins in LDS
  constexpr bool kPairs = kMode == 0 && kBqLds;
  __shared__ double s_yl[kPairs ? U * 256 : 1];

  const int b = blockIdx.x / bpi;
  const int blk = blockIdx.x - b * bpi;
  const int tid = threadIdx.x;
  const int N = a.N, n = a.n, H = n - U;
  if (kBqLds) {
    for (int e = tid; e < NB * kQ; e += 256) {
      const int k = e / kQ;
      s_bq[e] = lzq[((size_t)b * kMaxBeta + k) * lz_q_stride(U) + (e - k * kQ)];
    }
  }
  const int64_t lane = (int64_t)blk * 256 + tid;
  const bool valid = lane < a.lanes;
  const uint64_t p = valid ? (uint64_t)lane : 0ull;
  const float* Jt = J + (size_t)b * N * N;
  const float* ht = h + (size_t)b * N;
  const double* tab = table64 + ((size_t)b * a.table_recs + (size_t)a.table_offset) * (2 + U);

  // ---- per-lane init (fp64): y_f = sum_q J_fq s_q, the field on free spin f
  // from the prefix spins q >= n; E_P the energy of the prefix spins alone
  double y[U];
#pragma unroll
  for (int f = 0; f < U; ++f) {
    double acc = 0.0;
    for (int q = n; q < N; ++q) {
      const double jq = (double)Jt[f * N + q];
      acc += ((p >> (q - n)) & 1ull) ? jq : -jq;
    }
    y[f] = acc;
    if (kPairs) s_yl[f * 256 + tid] = acc;
  }
  for (int f = U; f < n; ++f) {
    double acc = 0.0;
    for (int q = n; q < N; ++q) {
      const double jq = (double)Jt[f * N + q];
      acc += ((p >> (q - n)) & 1ull) ? jq : -jq;
    }
    s_y[(f - U) * 256 + tid] = acc;
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
  // E_P - sum_{f<U} s_f y_f at a block start: low spins all -1, except spin
  // U-1 = +1 in odd blocks
  double ylo = 0.0;
#pragma unroll
  for (int f = 0; f < U - 1; ++f) ylo += y[f];
  const double epa0 = EP + ylo + y[U - 1], epa1 = EP + ylo - y[U - 1];
  const double base = lzqmin[b] - (double)a.e0[b];

  double c2[NB];   // -beta / ln 2
  float c2f2[NB];  // 2 c2, for the factor exponents
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    c2[k] = -(double)a.beta[k] * 1.4426950408889634;
    c2f2[k] = (float)(2.0 * c2[k]);
  }

  // per-lane totals
  double L[NB];                                 // forward
#pragma unroll
  for (int k = 0; k < NB; ++k) L[k] = 0.0;
  double Om = 0.0, A[U], M[kLzHigh];            // backward
#pragma unroll
  for (int f = 0; f < U; ++f) A[f] = 0.0;
#pragma unroll
  for (int k = 0; k < kLzHigh; ++k) M[k] = 0.0;
  // distributed free x free slots of this lane
  const int ln = tid & 63, wv = tid >> 6;
  const int nslots = 15 + U * H + H * (H - 1) / 2;
  int sc[2] = {0, 0}, st[2] = {0, 0};  // st: set-up only (targets are formed again at the end)
  uint32_t sm[2] = {0u, 0u};
  double dacc[2] = {0.0, 0.0};
  if (kMode == 1) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
      if (ln + 64 * r < nslots) lz_slot(ln + 64 * r, H, N, &sc[r], &sm[r], &st[r]);
  }
  __syncthreads();  // s_y, s_bq

  // field energy of the high spins, -sum_k s_k y_(U+k), all down at T = 0;
  // updated by one flip per block (fp64, at most 2^H - 1 terms)
  double gh = 0.0;
  for (int k = 0; k < H; ++k) gh += s_y[k * 256 + tid];

  const uint32_t nblocks = 1u << (n - U);
  // Records of 10 (bq in LDS): the blocks go in pairs (T, T + 1) and every
  // bq entry read from LDS enters the contractions of both.  A broadcast
  // read of four entries occupies the LDS for four cycles, once per four
  // fused multiply-adds of one block: with one block per read the LDS was
  // the bound (busy nine cycles in ten), not the VALU.
  // Block T's lower bound Lb of E - E0 over its configurations and the
  // coefficients phi_f of its low spins (fp32: only their magnitudes and
  // signs enter the factors), ghT being the high spins' field energy there.
  auto block_consts = [&](uint32_t T, double ghT, double& Lb, float (&ph)[U]) {
    const double* rec = tab + (size_t)T * (2 + U);
    const bool odd = T & 1u;
    // energy at the block start without the low-low part
    const double G0 = (odd ? epa1 : epa0) + rec[1] + ghT;
    double phi[U];
#pragma unroll
    for (int f = 0; f < U; ++f) {
      const double yf = kPairs ? s_yl[f * 256 + tid] : y[f];
      const double wf = f < U - 1 || odd ? rec[2 + f] : -rec[2 + f];
      phi[f] = -(yf + 0.5 * wf);
    }
    double K = odd ? G0 - phi[U - 1] : G0 + phi[U - 1];
    double sabs = 0.0;
#pragma unroll
    for (int f = 0; f < U; ++f) {
      if (f < U - 1) K += phi[f];
      sabs += fabs(phi[f]);
      ph[f] = (float)phi[f];
    }
    Lb = K - sabs + base;
  };
  // one flip of a high spin from block T - 1 to block T (T > 0)
  auto step_gh = [&](uint32_t T) {
    const uint32_t xh = T ^ (T >> 1);
    const int kb = __builtin_ctz(T);
    const double yb = 2.0 * s_y[kb * 256 + tid];
    gh = ((xh >> kb) & 1u) ? gh - yb : gh + yb;
  };
  // c_f(s_f) at beta k: 1 for the sign that lowers phi_f s_f, 2^(2 c2 |phi_f|)
  // for the other (cp: s_f = +1, cm: s_f = -1)
  auto factors = [&](int k, const float (&ph)[U], float* cp, float* cm) {
#pragma unroll
    for (int f = 0; f < U; ++f) {
      const float af = __builtin_amdgcn_exp2f(c2f2[k] * fabsf(ph[f]));
      cp[f] = ph[f] > 0.0f ? af : 1.0f;
      cm[f] = ph[f] > 0.0f ? 1.0f : af;
    }
  };
  if constexpr (kPairs) {
    for (uint32_t T = 0; T < nblocks; T += 2) {
      asm volatile("" ::: "memory");
      // a lane of a single block (n = U) gives the second block zero weight
      const bool two = T + 1 < nblocks;
      double Lb0, Lb1;
      float ph0[U], ph1[U];
      if (T) step_gh(T);
      block_consts(T, gh, Lb0, ph0);
      if (two) step_gh(T + 1);
      block_consts(two ? T + 1 : T, gh, Lb1, ph1);
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const double P0 = valid ? exp2_wide(c2[k] * Lb0) : 0.0;
        const double P1 = valid && two ? exp2_wide(c2[k] * Lb1) : 0.0;
        // A: the factor products of spins 0-4; B(r) for spins 5-9 is
        // B4(spins 5, 6) x B8(spins 7-9), applied to the row sums in two steps
        float cp[U], cm[U], A0[kM], A1[kM], B40[4], B41[4], B80[8], B81[8];
        factors(k, ph0, cp, cm);
        factor_products<U / 2>(cp, cm, A0);
        factor_products<2>(cp + U / 2, cm + U / 2, B40);
        factor_products<3>(cp + U / 2 + 2, cm + U / 2 + 2, B80);
        factors(k, ph1, cp, cm);
        factor_products<U / 2>(cp, cm, A1);
        factor_products<2>(cp + U / 2, cm + U / 2, B41);
        factor_products<3>(cp + U / 2 + 2, cm + U / 2 + 2, B81);
        // bq by configuration (x = x_lo + 2^(U/2) r) in chunks of kC
        // entries, each read one chunk ahead of its products; the empty asm
        // after each chunk keeps later chunks from being fetched early
        const float* q = s_bq + k * kQ;
        constexpr int kC = 8;
        constexpr int kPer = kM / kC;  // chunks per row
        float qc[kC], qn[kC];
#pragma unroll
        for (int i = 0; i < kC; ++i) qc[i] = q[i];
        float S0 = 0.0f, S1 = 0.0f, W0 = 0.0f, W1 = 0.0f, u0 = 0.0f, u1 = 0.0f;
#pragma unroll
        for (int c = 0; c < kM * kPer; ++c) {
          if (c + 1 < kM * kPer) {
#pragma unroll
            for (int i = 0; i < kC; ++i) qn[i] = q[kC * (c + 1) + i];
          }
          const int x1 = kC * (c % kPer);
#pragma unroll
          for (int i = 0; i < kC; ++i) {
            u0 = fmaf(A0[x1 + i], qc[i], u0);
            u1 = fmaf(A1[x1 + i], qc[i], u1);
          }
          if (c % kPer == kPer - 1) {
            const int r = c / kPer;
            W0 = fmaf(B40[r & 3], u0, W0);
            W1 = fmaf(B41[r & 3], u1, W1);
            u0 = 0.0f;
            u1 = 0.0f;
            if ((r & 3) == 3) {
              S0 = fmaf(B80[r >> 2], W0, S0);
              S1 = fmaf(B81[r >> 2], W1, S1);
              W0 = 0.0f;
              W1 = 0.0f;
            }
          }
          asm volatile("" : "+v"(S0), "+v"(S1), "+v"(W0), "+v"(W1), "+v"(u0), "+v"(u1) : : "memory");
#pragma unroll
          for (int i = 0; i < kC; ++i) qc[i] = qn[i];
        }
        L[k] += P0 * (double)S0 + P1 * (double)S1;
      }
    }
  } else {
    for (uint32_t T = 0; T < nblocks; ++T) {
      // the bq tables are re-read from LDS every block instead of being held in
      // registers for the whole lane
      asm volatile("" ::: "memory");
      const bool odd = T & 1u;
      const uint32_t xh = T ^ (T >> 1);  // high spins of this block (bit k: spin U + k)
      if (T) step_gh(T);
      double Lb;
      float ph[U];
      block_consts(T, gh, Lb, ph);
      // the gradient walk indexes spin U-1 by the bits of its Gray steps, which
      // flip that spin in odd blocks: exchange its two factors there
      if (kMode == 1 && odd) ph[U - 1] = -ph[U - 1];

      if constexpr (kMode == 0) {
        // one beta at a time: sum_x A(x_lo) B(x_hi) bq(x) over the 2^U
        // configurations, x_lo the spins below U/2
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const double P = valid ? exp2_wide(c2[k] * Lb) : 0.0;
          float cp[U], cm[U], Af[kM], Bf[kM];
          factors(k, ph, cp, cm);
          factor_products<U / 2>(cp, cm, Af);
          factor_products<U / 2>(cp + U / 2, cm + U / 2, Bf);
          // bq by configuration (wave-uniform: scalar loads into SGPRs for
          // blocks of 8, broadcast LDS reads for blocks of 10), in chunks of
          // kC = min(2^(U/2), 16) entries, each read one chunk ahead of its
          // products.  The empty asm after each chunk ties its products
          // (through u) to the reads (memory clobber), so later chunks are not
          // fetched early.
          const float* q =
              kBqLds ? s_bq + k * kQ : lzq + ((size_t)b * kMaxBeta + k) * lz_q_stride(U);
          constexpr int kC = kM < 16 ? kM : 16;
          constexpr int kPer = kM / kC;  // chunks per row
          float qc[kC], qn[kC];
#pragma unroll
          for (int i = 0; i < kC; ++i) qc[i] = q[i];
          float S = 0.0f, u = 0.0f;
#pragma unroll
          for (int c = 0; c < kM * kPer; ++c) {
            if (c + 1 < kM * kPer) {
#pragma unroll
              for (int i = 0; i < kC; ++i) qn[i] = q[kC * (c + 1) + i];
            }
            const int x1 = kC * (c % kPer);
#pragma unroll
            for (int i = 0; i < kC; ++i) u = fmaf(Af[x1 + i], qc[i], u);
            if (c % kPer == kPer - 1) {
              S = fmaf(Bf[c / kPer], u, S);
              u = 0.0f;
            }
            asm volatile("" : "+v"(S), "+v"(u) : : "memory");
#pragma unroll
            for (int i = 0; i < kC; ++i) qc[i] = qn[i];
          }
          L[k] += P * (double)S;
        }
      } else {
        // A: factor products of spins 0-2 times the beta's weight (folded into
        // spin 0's two factors); B: spins 3-5, indexed by the Gray step's bits
        // (block parity folded in through up[])
        float Af[NB][8], Bf[NB][8];
        const float* bqs[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const double P = valid ? exp2_wide(c2[k] * Lb) : 0.0;
          const float sk = (float)(a.coef[(size_t)b * 2 * kMaxBeta + k] * P);
          float cp[U], cm[U];
          factors(k, ph, cp, cm);
          cp[0] *= sk;
          cm[0] *= sk;
          factor_products<3>(cp, cm, Af[k]);
          factor_products<3>(cp + 3, cm + 3, Bf[k]);
          bqs[k] = s_bq + k * kQ + kSteps * (odd ? 2 : 1);
        }
        BlockWalk<NB, false> bw{Af, Bf, bqs, nullptr, odd ? 1.0f : -1.0f};
        const Coefs C = bw.template walk<U, 0>();
        // per-lane totals for the prefix-involving moments
        Om += (double)C.o;
#pragma unroll
        for (int f = 0; f < U; ++f) A[f] += (double)C.s[f];
#pragma unroll
        for (int k = 0; k < kLzHigh; ++k)
          if (k < H) M[k] += ((xh >> k) & 1u) ? (double)C.o : -(double)C.o;
        // wave sums of the 22 coefficients: each is first summed over the 16
        // lanes of its row by DPP shifts (the row's last lane ends with the
        // total), the 4 row totals go through LDS (one 24-float row each), and
        // lane c < 22 adds the four totals of coefficient c
        float cv[kCoefStride];
        cv[0] = row_total(C.o);
#pragma unroll
        for (int f = 0; f < U; ++f) cv[1 + f] = row_total(C.s[f]);
#pragma unroll
        for (int k = 0; k < 15; ++k) cv[1 + U + k] = row_total(C.p[k]);
        cv[kNCoef] = 0.0f;
        cv[kNCoef + 1] = 0.0f;
        if ((ln & 15) == 15) {
          float* cw = s_c + (wv * 4 + (ln >> 4)) * kCoefStride;
#pragma unroll
          for (int j = 0; j < kCoefStride; j += 4)
            *(float4*)(cw + j) = make_float4(cv[j], cv[j + 1], cv[j + 2], cv[j + 3]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (ln < kNCoef) {
          const float* col = s_c + wv * 4 * kCoefStride + ln;
          s_t[wv * kNCoef + ln] = (col[0] + col[kCoefStride]) +
                                  (col[2 * kCoefStride] + col[3 * kCoefStride]);
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
  }

  // ---- lane end: reduce over the lanes of the wave, one atomic per value
  double* acc = a.acc + (size_t)b * a.acc_stride;
  const bool lead = ln == 0;
  if (kMode == 0) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const double t = wave_sum(L[k]);
      if (lead) atomicAdd(acc + k, t);
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
  // free x free pairs from the distributed slots (their targets are formed
  // again here rather than carried through the walk)
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    if (ln + 64 * r < nslots) {
      int c2 = 0, t2 = 0;
      uint32_t m2 = 0u;
      lz_slot(ln + 64 * r, H, N, &c2, &m2, &t2);
      atomicAdd(acc + t2, dacc[r]);
    }
  }
}

// ------------------------------------------- gradient walk over records of 8
// The records of kLzUF = 8 low spins (those of the partition sums): spins
// 8..n-1 are fixed per record T, and the record is walked as four sub-blocks
// of the 64 configurations of spins 0..5, sub-block j with spins 6 and 7 set
// to gray2(j).  Within the record
//   E(x) = K_T + sum_{f<8} phi_f s_f + Q8(x),
// Q8 the energy of the couplings among spins 0..7, so a sub-block's combined
// weights are
//   omega(x) = sum_b coef_b P_T,b prod_{f<6} c_f(s_f) * c_6(s_6) c_7(s_7) * bq8_b(x)
// with bq8_b(x) = exp(-beta_b (Q8(x) - min Q8)) tabulated by sub-block and
// Gray step.  The record's bound, its 24 exponentials and the factor tables
// are formed once per 256 configurations; a sub-block scales B (spins 3-5) by
// its factors of spins 6 and 7.  Walsh coefficients, slots and per-lane totals
// are those of the blocks of 6, spins 6 and 7 counting as high spins.

// A wave-uniform value in scalar registers.
__device__ inline float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ inline double uniform_d(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Wave sums of the 22 block coefficients v[0..21].  v_permlane32_swap trades
// the upper half-wave of coefficient i for the lower half-wave of i + 11, so
// one add leaves each lane the sum of lanes l and l ^ 32 of one of the two;
// v_permlane16_swap does the same between rows for i and i + 5 of the 11
// left (the last one with itself); each lane then holds 6 sums of 4 lanes,
// and DPP row shifts finish the row totals in each row's last lane.  Which
// coefficient a row's u[i] totals follows from the same exchanges applied to
// the coefficient numbers (coef_rows), so nothing here depends on which half
// of a swap moves which way: row r ends with coefficients c_r + i (i < 5) and
// one of the two unpaired ones in u[5].
__device__ inline void coef_wave_sums(const float* v, float* u) {
  float w[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]),
                                                    __float_as_uint(v[i + 11]), false, false);
    w[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float x = w[i], z = i < 5 ? w[i + 5] : w[10];
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(i < 5 ? x : z),
                                                    __float_as_uint(z), false, false);
    u[i] = row_total(__uint_as_float(r[0]) + __uint_as_float(r[1]));
  }
}

// Coefficient numbers of a lane's u[0] and u[5] after coef_wave_sums.
__device__ inline void coef_rows(int* c0, int* c5) {
  int w[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap((uint32_t)i, (uint32_t)(i + 11), false, false);
    w[i] = (int)r[0];
  }
  const auto r0 = __builtin_amdgcn_permlane16_swap((uint32_t)w[0], (uint32_t)w[5], false, false);
  const auto r5 = __builtin_amdgcn_permlane16_swap((uint32_t)w[10], (uint32_t)w[10], false, false);
  *c0 = (int)r0[0];
  *c5 = (int)r5[0];
}

template <int NB>
__global__ __launch_bounds__(256, (lz_min_blocks<1, NB>())) void k_lz_grad8(
    LzArgs a, const float* __restrict__ J, const float* __restrict__ h,
    const double* __restrict__ table64, const float* __restrict__ lzq,
    const double* __restrict__ lzqmin, int bpi) {
  constexpr int U = kLzUF;                 // spins per record
  constexpr int V = kLzU;                  // spins per sub-block (the Walsh tree's)
  constexpr int kSub = 1 << (U - V);       // sub-blocks per record
  constexpr int kQ = lz_q_floats<1, U>();  // bq floats per beta
  static_assert(kQ == kSub * (1 << V), "one bq row of 64 per sub-block");
  __shared__ double s_y[kLzFree * 256];  // y_f of every free spin, read per record
  __shared__ double s_m[kLzHigh * 256];  // per-lane totals M_k of the high spins
  __shared__ float s_t[4 * kNCoef];

  const int b = blockIdx.x / bpi;
  const int blk = blockIdx.x - b * bpi;
  const int tid = threadIdx.x;
  const int N = a.N, n = a.n, H = n - V;  // H: high spins 6..n-1 of the slots
  const int64_t lane = (int64_t)blk * 256 + tid;
  const bool valid = lane < a.lanes;
  const uint64_t p = valid ? (uint64_t)lane : 0ull;
  const float* Jt = J + (size_t)b * N * N;
  const float* ht = h + (size_t)b * N;
  const double* tab = table64 + ((size_t)b * a.table_recs + (size_t)a.table_offset) * (2 + U);

  // ---- per-lane init (fp64): y_f = sum_q J_fq s_q, the field on free spin f
  // from the prefix spins; E_P the energy of the prefix spins alone
  double ysum = 0.0, y7 = 0.0;  // sum_{f<7} y_f, y_7
  for (int f = 0; f < n; ++f) {
    double acc = 0.0;
    for (int q = n; q < N; ++q) {
      const double jq = (double)Jt[f * N + q];
      acc += ((p >> (q - n)) & 1ull) ? jq : -jq;
    }
    s_y[f * 256 + tid] = acc;
    if (f < U - 1) ysum += acc;
    if (f == U - 1) y7 = acc;
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
  // E_P - sum_{f<8} s_f y_f at a record start: spins 0..6 down, spin 7 up in
  // odd records
  const double epa0 = EP + ysum + y7, epa1 = EP + ysum - y7;
  const double base = uniform_d(lzqmin[b] - (double)a.e0[b]);

  // per-beta constants, loaded (not computed) so that they stay in scalar
  // registers
  const double* cb = a.coef + (size_t)b * 2 * kMaxBeta;
  double c2[NB];   // -beta / ln 2
  float c2f2[NB];  // 2 c2, for the factor exponents
  double cf[NB];   // the beta's gradient weight
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    c2[k] = cb[kMaxBeta + k];
    c2f2[k] = uniform_f((float)(2.0 * c2[k]));
    cf[k] = cb[k];
  }

  // per-lane totals for the prefix-involving moments (M_k in LDS, updated
  // once per record)
  double Om = 0.0, A[V];
#pragma unroll
  for (int f = 0; f < V; ++f) A[f] = 0.0;
#pragma unroll
  for (int k = 0; k < kLzHigh; ++k) s_m[k * 256 + tid] = 0.0;
  // distributed free x free slots of this lane
  const int ln = tid & 63, wv = tid >> 6;
  const int nslots = 15 + V * H + H * (H - 1) / 2;
  int sc[2] = {0, 0};
  uint32_t sm[2] = {0u, 0u};
  double dacc[2] = {0.0, 0.0};
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    int t = 0;
    if (ln + 64 * r < nslots) lz_slot(ln + 64 * r, H, N, &sc[r], &sm[r], &t);
  }
  // where a row's last lane leaves its coefficient totals
  int c0 = 0, c5 = 0;
  coef_rows(&c0, &c5);
  float* const t0 = s_t + wv * kNCoef + c0;
  float* const t5 = s_t + wv * kNCoef + c5;
  const bool row_end = (ln & 15) == 15;
  // field energy of the high spins 8..n-1, -sum_k s_k y_(8+k), all down at
  // T = 0; updated by one flip per record (fp64, at most 2^(n-8) - 1 terms)
  double gh = 0.0;
  for (int k = U; k < n; ++k) gh += s_y[k * 256 + tid];

  const uint32_t nrec = 1u << (n - U);
  for (uint32_t T = 0; T < nrec; ++T) {
    const double* rec = tab + (size_t)T * (2 + U);
    const bool odd = T & 1u;
    const uint32_t x8 = T ^ (T >> 1);  // spins 8.. of this record (bit k: spin 8 + k)
    if (T) {
      const int kb = __builtin_ctz(T);  // the spin that flipped
      const double yb = 2.0 * s_y[(U + kb) * 256 + tid];
      gh = ((x8 >> kb) & 1u) ? gh - yb : gh + yb;
    }
    // energy at the record start without the low-low part
    const double G0 = (odd ? epa1 : epa0) + rec[1] + gh;
    double phi[U];
#pragma unroll
    for (int f = 0; f < U - 1; ++f) phi[f] = -(s_y[f * 256 + tid] + 0.5 * rec[2 + f]);
    phi[U - 1] = -(s_y[(U - 1) * 256 + tid] + 0.5 * (odd ? rec[2 + U - 1] : -rec[2 + U - 1]));
    double K = odd ? G0 - phi[U - 1] : G0 + phi[U - 1];
    double sabs = 0.0;
#pragma unroll
    for (int f = 0; f < U; ++f) {
      if (f < U - 1) K += phi[f];
      sabs += fabs(phi[f]);
    }
    const double Lb = K - sabs + base;  // lower bound of E - E0 over the record

    // factors: c_f(s_f) at beta k is 1 for the sign that lowers phi_f s_f,
    // 2^(2 c2 |phi_f|) for the other
    // spins 6 and 7: a6, a7 their non-1 factors, costly when up (the sign
    // that raises phi_f s_f is +1) or down
    float Af[NB][8], Bf[NB][8], a6[NB], a7[NB];
    const bool hi6 = phi[6] > 0.0, hi7 = phi[7] > 0.0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const double P = valid ? exp2_wide(c2[k] * Lb) : 0.0;
      const float sk = (float)(cf[k] * P);
      float cp[U], cm[U];
#pragma unroll
      for (int f = 0; f < U; ++f) {
        const float af = __builtin_amdgcn_exp2f(c2f2[k] * (float)fabs(phi[f]));
        const bool up = phi[f] > 0.0;
        cp[f] = up ? af : 1.0f;
        cm[f] = up ? 1.0f : af;
      }
      cp[0] *= sk;
      cm[0] *= sk;
      factor_products<3>(cp, cm, Af[k]);
      factor_products<3>(cp + 3, cm + 3, Bf[k]);
      a6[k] = hi6 ? cp[6] : cm[6];
      a7[k] = hi7 ? cp[7] : cm[7];
    }

    float om_r = 0.0f, a_r[V], m6 = 0.0f, m7 = 0.0f;  // record partial sums
#pragma unroll
    for (int f = 0; f < V; ++f) a_r[f] = 0.0f;
#pragma nounroll
    for (int j = 0; j < kSub; ++j) {
      // the sub-block's bq rows are wave-uniform: scalar loads into SGPRs,
      // issued per sub-block (the memory clobber keeps them from being
      // hoisted out of the loop)
      asm volatile("" ::: "memory");
      const int gj = j ^ (j >> 1);  // bit 0: spin 6 up, bit 1: spin 7 up
      const bool up6 = gj & 1, up7 = gj & 2;
      const bool x6 = up6 == hi6, x7 = up7 == hi7;  // spin 6 (7) takes its factor
      float d[NB];
      const float* bqs[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        d[k] = (x6 ? a6[k] : 1.0f) * (x7 ? a7[k] : 1.0f);
        bqs[k] = lzq + ((size_t)b * kMaxBeta + k) * lz_q_stride(U) + j * (1 << V);
      }
      BlockWalk<NB, true> bw{Af, Bf, bqs, d, 0.0f};
      const Coefs C = bw.template walk<V, 0>();
      om_r += C.o;
#pragma unroll
      for (int f = 0; f < V; ++f) a_r[f] += C.s[f];
      m6 += up6 ? C.o : -C.o;
      m7 += up7 ? C.o : -C.o;
      // wave sums of the 22 coefficients, then the slots' signed sums
      float v[kNCoef], u[6];
      v[0] = C.o;
#pragma unroll
      for (int f = 0; f < V; ++f) v[1 + f] = C.s[f];
#pragma unroll
      for (int k = 0; k < 15; ++k) v[1 + V + k] = C.p[k];
      coef_wave_sums(v, u);
      if (row_end) {
#pragma unroll
        for (int i = 0; i < 5; ++i) t0[i] = u[i];
        *t5 = u[5];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const uint32_t xh = (uint32_t)gj | (x8 << 2);  // bit k: spin 6 + k
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        if (ln + 64 * r < nslots) {
          const float tv = s_t[wv * kNCoef + sc[r]];
          // product of the high signs in the mask: -1 per high spin that is down
          const int downs = __popc(sm[r]) - __popc(sm[r] & xh);
          dacc[r] += (downs & 1) ? -(double)tv : (double)tv;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    Om += (double)om_r;
#pragma unroll
    for (int f = 0; f < V; ++f) A[f] += (double)a_r[f];
    s_m[tid] += (double)m6;
    s_m[256 + tid] += (double)m7;
#pragma unroll
    for (int k = 2; k < kLzHigh; ++k)
      if (k < H) s_m[k * 256 + tid] += ((x8 >> (k - 2)) & 1u) ? (double)om_r : -(double)om_r;
  }

  // ---- lane end: reduce over the lanes of the wave, one atomic per value
  double* acc = a.acc + (size_t)b * a.acc_stride;
  const bool lead = ln == 0;
  auto sp = [&](int q) -> double { return ((p >> (q - n)) & 1ull) ? 1.0 : -1.0; };
#pragma unroll
  for (int f = 0; f < V; ++f) {
    const double t = wave_sum(A[f]);
    if (lead) atomicAdd(acc + N * N + f, t);
  }
  double M[kLzHigh];
#pragma unroll
  for (int g = 0; g < kLzHigh; ++g) {
    M[g] = s_m[g * 256 + tid];
    if (g < H) {
      const double t = wave_sum(M[g]);
      if (lead) atomicAdd(acc + N * N + V + g, t);
    }
  }
  for (int q = n; q < N; ++q) {
    const double sq = sp(q);
    double t = wave_sum(sq * Om);
    if (lead) atomicAdd(acc + N * N + q, t);
    for (int r = q + 1; r < N; ++r) {
      t = wave_sum(sq * sp(r) * Om);
      if (lead) atomicAdd(acc + q * N + r, t);
    }
#pragma unroll
    for (int f = 0; f < V; ++f) {
      t = wave_sum(sq * A[f]);
      if (lead) atomicAdd(acc + f * N + q, t);
    }
#pragma unroll
    for (int g = 0; g < kLzHigh; ++g) {
      if (g < H) {
        t = wave_sum(sq * M[g]);
        if (lead) atomicAdd(acc + (V + g) * N + q, t);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    if (ln + 64 * r < nslots) {
      int c = 0, t = 0;
      uint32_t m = 0u;
      lz_slot(ln + 64 * r, H, N, &c, &m, &t);
      atomicAdd(acc + t, dacc[r]);
    }
  }
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

hipError_t launch_lz_prep(int mode, const LzArgs& a, const float* J, float* lzq, double* lzqmin,
                          const float* energies, float* e0_out, const double* logz,
                          const double* grad, hipStream_t st) {
  if (mode == 0 && a.U == kLzUW)
    hipLaunchKernelGGL((k_lz_prep<0, kLzUW>), dim3(a.B), dim3(256), 0, st, a, J, lzq, lzqmin,
                       energies, e0_out, logz, grad);
  else if (mode == 0 && a.U == kLzUF)
    hipLaunchKernelGGL((k_lz_prep<0, kLzUF>), dim3(a.B), dim3(256), 0, st, a, J, lzq, lzqmin,
                       energies, e0_out, logz, grad);
  else if (mode == 0 && a.U == kLzU)
    hipLaunchKernelGGL((k_lz_prep<0, kLzU>), dim3(a.B), dim3(256), 0, st, a, J, lzq, lzqmin,
                       energies, e0_out, logz, grad);
  else if (mode == 1 && a.U == kLzU)
    hipLaunchKernelGGL((k_lz_prep<1, kLzU>), dim3(a.B), dim3(256), 0, st, a, J, lzq, lzqmin,
                       energies, e0_out, logz, grad);
  else if (mode == 1 && a.U == kLzUF)
    hipLaunchKernelGGL((k_lz_prep<1, kLzUF>), dim3(a.B), dim3(256), 0, st, a, J, lzq, lzqmin,
                       energies, e0_out, logz, grad);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_logz(int mode, const LzArgs& a, const float* J, const float* h,
                       const double* table64, const float* lzq, const double* lzqmin,
                       hipStream_t st) {
  const int bpi = (int)((a.lanes + 255) / 256);
  const dim3 grid((unsigned)((int64_t)bpi * a.B));
#define SG_LZ_LAUNCH(M, NBV, UV)                                                          \
  hipLaunchKernelGGL((k_logz<M, NBV, UV>), grid, dim3(256), 0, st, a, J, h, table64, lzq, lzqmin, \
                     bpi)
  if (mode == 1 && a.U == kLzUF) {
#define SG_LZ8_LAUNCH(NBV)                                                                 \
  hipLaunchKernelGGL((k_lz_grad8<NBV>), grid, dim3(256), 0, st, a, J, h, table64, lzq, lzqmin, bpi)
    switch (a.nb) {
      case 1: SG_LZ8_LAUNCH(1); break;
      case 2: SG_LZ8_LAUNCH(2); break;
      case 3: SG_LZ8_LAUNCH(3); break;
      case 4: SG_LZ8_LAUNCH(4); break;
      default: return hipErrorInvalidValue;
    }
#undef SG_LZ8_LAUNCH
  } else if (mode == 0 && a.U == kLzUW) {
    switch (a.nb) {
      case 1: SG_LZ_LAUNCH(0, 1, kLzUW); break;
      case 2: SG_LZ_LAUNCH(0, 2, kLzUW); break;
      case 3: SG_LZ_LAUNCH(0, 3, kLzUW); break;
      default: return hipErrorInvalidValue;  // four beta take records of 8
    }
  } else if (mode == 0 && a.U == kLzUF) {
    switch (a.nb) {
      case 1: SG_LZ_LAUNCH(0, 1, kLzUF); break;
      case 2: SG_LZ_LAUNCH(0, 2, kLzUF); break;
      case 3: SG_LZ_LAUNCH(0, 3, kLzUF); break;
      case 4: SG_LZ_LAUNCH(0, 4, kLzUF); break;
      default: return hipErrorInvalidValue;
    }
  } else if (a.U == kLzU) {
    switch (mode * 8 + a.nb) {
      case 1: SG_LZ_LAUNCH(0, 1, kLzU); break;
      case 2: SG_LZ_LAUNCH(0, 2, kLzU); break;
      case 3: SG_LZ_LAUNCH(0, 3, kLzU); break;
      case 4: SG_LZ_LAUNCH(0, 4, kLzU); break;
      case 9: SG_LZ_LAUNCH(1, 1, kLzU); break;
      case 10: SG_LZ_LAUNCH(1, 2, kLzU); break;
      case 11: SG_LZ_LAUNCH(1, 3, kLzU); break;
      case 12: SG_LZ_LAUNCH(1, 4, kLzU); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
#undef SG_LZ_LAUNCH
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

// ------------------------------------------------------------ static scratch
// The allocation-free backward keeps its block records, bq tables, weights,
// accumulators and error word in this array instead of a workspace.  Every
// device holds its own copy from the library's load until the process ends;
// host code reaches it only through the device address that lz_scratch
// resolves (the array's name is a host-side stand-in there).

static __device__ __align__(256) unsigned char scratch[kLzScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device -> address of its scratch

__global__ void k_clear_word(uint32_t* p) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = 0u;
}

// Device address of the current device's scratch; *fresh is set on the call
// that resolves it (once per device), after which the caller clears the
// array's error word.
hipError_t lz_scratch(void** ptr, bool* fresh) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *ptr = it->second;
    *fresh = false;
    return hipSuccess;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[dev] = p;
  *ptr = p;
  *fresh = true;
  return hipSuccess;
}

// The current device's scratch address if it was resolved, else null.
void* lz_scratch_resolved() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  return it == g_scratch_addr.end() ? nullptr : it->second;
}

hipError_t launch_clear_word(uint32_t* p, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, st, p);
  return hipGetLastError();
}

}  // namespace sg
