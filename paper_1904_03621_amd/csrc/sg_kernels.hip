// sg_kernels.hip -- gfx950 kernels of the exhaustive low-spectrum search.
//
// Pipeline of one search over B instances (B = 1 for a single instance), all
// on one stream with no host round trip:
//   k_prep       per-instance checks, |J|+|h| bound, pruning margin, Q tables
//   k_tables     per-block records of every free-spin count n in use
//   per chunk of the state space (Sec. 3, Algorithm 1):
//     k_enum     Gray-code enumeration, one lane per prefix; candidates out
//     k_score +  exact energy of every candidate, keep those beating the
//     k_merge    current S-th key, sort them and merge them into the running
//                top-S record (single instance: a grid + one workgroup;
//                batch: k_merge_batched, one workgroup per instance)
//   k_finalize   record -> caller's output arrays
//
// Energy of Eq. (1), mask bit i <-> spin i, bit set <-> s_i = +1.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_internal.h"

namespace sg {

// ------------------------------------------------------------------ helpers

__device__ inline int inst_N(const Batch& bt, int b) { return bt.Ns ? bt.Ns[b] : bt.N0; }

template <typename T>
__device__ inline const T* inst_J(const Batch& bt, int b) {
  return (const T*)bt.J + (size_t)b * bt.ld * bt.ld;
}
template <typename T>
__device__ inline const T* inst_h(const Batch& bt, int b) {
  return (const T*)bt.h + (size_t)b * bt.ld;
}

__device__ inline uint32_t gray32(uint32_t t) { return t ^ (t >> 1); }

// Energy of one state from scratch, Eq. (1), fixed i<j order; J has row
// stride ld.  A row's couplings are read eight at a time before they are
// summed (in the same order), so the reads overlap instead of each waiting
// on the previous add; s_j J_ij is formed as +-J_ij (exact).
__device__ inline double energy_f64(const float* J, const float* h, int N, int ld, uint64_t m) {
  double e = 0.0;
  for (int i = 0; i < N; ++i) {
    const float* row = J + i * ld;
    double f = (double)h[i];
    int j = i + 1;
    for (; j + 8 <= N; j += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = row[j + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) f += ((m >> (j + u)) & 1ull) ? (double)v[u] : -(double)v[u];
    }
    for (; j < N; ++j) f += ((m >> j) & 1ull) ? (double)row[j] : -(double)row[j];
    e -= ((m >> i) & 1ull) ? f : -f;
  }
  return e;
}

__device__ inline int32_t energy_i32(const int32_t* J, const int32_t* h, int N, int ld,
                                     uint64_t m) {
  int32_t e = 0;
  for (int i = 0; i < N; ++i) {
    const int32_t* row = J + i * ld;
    int32_t f = h[i];
    int j = i + 1;
    for (; j + 8 <= N; j += 8) {
      int32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = row[j + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) f += ((m >> (j + u)) & 1ull) ? v[u] : -v[u];
    }
    for (; j < N; ++j) f += ((m >> j) & 1ull) ? row[j] : -row[j];
    e -= ((m >> i) & 1ull) ? f : -f;
  }
  return e;
}

// float nearest to x from below / above (x finite)
__device__ inline float f32_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = __uint_as_float(f > 0.0f ? __float_as_uint(f) - 1u
                                          : (f == 0.0f ? 0x80000001u : __float_as_uint(f) + 1u));
  return f;
}
__device__ inline float f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = __uint_as_float(f < 0.0f ? __float_as_uint(f) - 1u
                                          : (f == 0.0f ? 0x00000001u : __float_as_uint(f) + 1u));
  return f;
}

__device__ inline uint32_t key_f32(float e) {
  if (e == 0.0f) e = 0.0f;  // -0 -> +0
  return key_of_f32_bits(__float_as_uint(e));
}

__device__ inline bool key_less(uint32_t ka, uint64_t ma, uint32_t kb, uint64_t mb) {
  return ka < kb || (ka == kb && ma < mb);
}

// ------------------------------------------------------------------ k_prep
// One workgroup per instance.  Writes the Q tables (low-spin coupling energy
// for both block parities) of both block sizes and their minima, the pruning
// margin, the error flags and the initial (empty) record state.

// Q(x) = -sum_{f<f'<U} J_ff' s_f s_f' over the low configuration
// x = gray(i) ^ (par << (U-1)) of step i in a block of parity par, written to
// qtab[par 2^U + i]; returns (to every thread) the minimum over both parities.
template <bool kInt, int U, typename T>
__device__ double prep_qtab(const T* Jb, int ld, int Nc, bool walk_f32, uint32_t* qtab,
                            double* s_q) {
  constexpr int kSteps = 1 << U;
  const int tid = threadIdx.x;
  for (int e = tid; e < 2 * kSteps; e += blockDim.x) {
    const int par = e / kSteps, i = e % kSteps;
    const uint32_t x = gray32((uint32_t)i) ^ ((uint32_t)par << (U - 1));
    double q = 0.0;
    for (int a = 0; a < U && a < Nc; ++a)
      for (int c = a + 1; c < U && c < Nc; ++c) {
        const double sa = ((x >> a) & 1u) ? 1.0 : -1.0, sc = ((x >> c) & 1u) ? 1.0 : -1.0;
        q -= (double)Jb[a * ld + c] * sa * sc;
      }
    s_q[e] = q;
    if (kInt && !walk_f32) qtab[e] = (uint32_t)(int32_t)q;
    else qtab[e] = __float_as_uint((float)q);
  }
  __syncthreads();
  // minimum: a strided pass down to 256 values, then halving
  if (2 * kSteps > 256) {
    double m0 = s_q[tid];
    for (int e = tid + 256; e < 2 * kSteps; e += 256) m0 = fmin(m0, s_q[e]);
    __syncthreads();
    s_q[tid] = m0;
    __syncthreads();
  }
  constexpr int kTop = 2 * kSteps > 256 ? 128 : kSteps;
  for (int st = kTop; st > 0; st >>= 1) {
    if (tid < st) s_q[tid] = fmin(s_q[tid], s_q[tid + st]);
    __syncthreads();
  }
  const double m = s_q[0];
  __syncthreads();  // s_q is reused
  return m;
}

template <bool kInt>
__global__ void k_prep(Batch bt) {
  const int b = blockIdx.x;
  const int N = inst_N(bt, b);
  const int ld = bt.ld;
  Params* P = bt.P + b;
  uint32_t* qtab = bt.qtab + (size_t)b * kQStride;
  // a batch (per-instance sizes) needs N_b >= U; a single search takes any N >= 1
  const bool badN = N < (bt.Ns ? kU : 1) || N > ld || (N < 63 && (uint64_t)bt.S > (1ull << N));
  const int Nc = badN ? 0 : N;
  using T = typename std::conditional<kInt, int32_t, float>::type;
  const T* Jb = inst_J<T>(bt, b);
  const T* hb = inst_h<T>(bt, b);

  __shared__ double s_sum[256];
  __shared__ int s_bad[256];
  __shared__ int s_lsb[256];
  const int tid = threadIdx.x;
  double acc = 0.0;
  int bad = 0;
  int lsb = 1 << 20;  // smallest exponent of a set bit over all values (fp32)
  for (int idx = tid; idx < Nc * Nc + Nc; idx += blockDim.x) {
    double v;
    bool use;
    if (idx < Nc * Nc) {
      const int i = idx / Nc, j = idx % Nc;
      use = i < j;
      v = (double)Jb[i * ld + j];
    } else {
      use = true;
      v = (double)hb[idx - Nc * Nc];
    }
    if (use) {
      if (!kInt && !isfinite(v)) bad = 1;
      else acc += fabs(v);
      if (!kInt && v != 0.0) {
        const uint32_t bits = __float_as_uint((float)v);
        const int ex = (int)((bits >> 23) & 0xffu);
        const uint32_t man = bits & 0x7fffffu;
        const int e = ex == 0 ? -149 + __builtin_ctz(man)
                              : ex - 150 + __builtin_ctz(man | 0x800000u);
        lsb = min(lsb, e);
      }
    }
  }
  s_sum[tid] = acc;
  s_bad[tid] = bad;
  s_lsb[tid] = lsb;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      s_sum[tid] += s_sum[tid + st];
      s_bad[tid] |= s_bad[tid + st];
      s_lsb[tid] = min(s_lsb[tid], s_lsb[tid + st]);
    }
    __syncthreads();
  }
  const double Bv = s_sum[0];
  const int anybad = s_bad[0];
  const int lsb_min = s_lsb[0];

  // An integer instance whose energies stay below 2^24 (2.1 Bv < 2^24: every
  // value on the walk is an integer of at most 24 bits) is walked in fp32,
  // where the walk is exact and, on this GPU, faster than in int32; its tables
  // then hold fp32 values.
  const bool walk_f32 = kInt && bt.allow_f32_walk && 2.1 * Bv < 16777216.0;
  // Q tables of both block sizes and their minima
  __shared__ double s_q[2 << kUPk];
  const double qmin7 = prep_qtab<kInt, kU>(Jb, ld, Nc, walk_f32, qtab + qtab_base(kU), s_q);
  const double qmin8 =
      prep_qtab<kInt, kUWide>(Jb, ld, Nc, walk_f32, qtab + qtab_base(kUWide), s_q);
  // blocks of kUPk: walks in fp32
  const bool pk10 = !kInt || walk_f32;
  const double qmin10 =
      pk10 ? prep_qtab<kInt, kUPk>(Jb, ld, Nc, walk_f32, qtab + qtab_base(kUPk), s_q) : 0.0;
  if (tid == 0) {
    uint32_t err = 0;
    if (badN) err |= kErrInval;
    if (anybad) err |= kErrNonFinite;
    if (kInt && Bv >= 268435456.0) err |= kErrOverflow;  // 2^28
    // Margin (fp32): a bound on |computed E - exact E| of any state, plus
    // the rounding of the rescored key.  Exact G, W, Y, the table constants
    // and energies are all bounded by 2 Bv; the computed ones stay below
    // 2 Bv + margin < 2.1 Bv (margin < 0.01 Bv below), so each fp32
    // rounding is at most uH = H 2^-24, H the power of two above 2.1 Bv.
    // Between two re-anchors (R = 2^10 / 2^U blocks) G takes per block 2^U - 1
    // rounded inner adds, 2 rounded boundary adds and a rounded boundary
    // constant, and the block's W values carry three roundings each with net
    // weight at most 1 per block (a spin's flips alternate in sign).  The
    // re-anchor itself rounds n + 3 times and starts from per-lane fields
    // rounded once each (n/2, fixed per lane: the high fields enter with net
    // weight <= 1 over any stretch); add the final E = G + Q (2) and the key
    // rounding (2).  When every value is a multiple of 2^lsb and 2.1 Bv
    // < 2^(24 + lsb), every fp32 operation on the path is exact: margin 0.
    double margin = 0.0;
    if (!kInt) {
      double H = 1.0;
      while (H <= 2.1 * Bv) H *= 2.0;
      const bool exact = Bv == 0.0 || (lsb_min < (1 << 19) && 2.1 * Bv < ldexp(1.0, 24 + lsb_min));
      if (!exact) {
        const double uH = H * 5.9604644775390625e-08;  // 2^-24
        // the larger count of the two block sizes (U = 7: 1208, U = 8: 1128)
        double walk = 0.0;
        for (int U = kU; U <= kUWide; ++U)
          walk = fmax(walk, (double)(1 << (kReanchorLog2 - U)) * ((1 << U) - 1.0 + 3.0 * U + 3.0));
        const double rounds = walk + (kMaxFree + 3.0) + kMaxFree * 0.5 + 4.0 + 4.0;
        margin = rounds * uH * (double)bt.margin_scale;
      }
    }
    // Paired walk (fp32 walks only): every field value is (G - fastThr) sc
    // + 2^15 - slack plus at most U + 1 units of rounding (the start value
    // and up to U low-spin steps of two roundings each), with
    // |G - fastThr| <= R = 2 Bv + 2 BQ + 2 margin + 1 (G = E - Q with
    // |E| <= Bv, |Q| <= BQ over the U low spins, walk values within the
    // margin); sc is the largest power of two with R sc + slack + U + 2
    // <= 2^15, so no field ever leaves [0, 2^16).  A slack of U + 1 units
    // keeps every state whose value is at or below fastThr below 2^15.
    auto pk_scale_of = [&](int U) -> float {
      if (!(!kInt || walk_f32) || anybad || badN) return 0.0f;
      double BQ = 0.0;
      for (int a = 0; a < U && a < Nc; ++a)
        for (int c = a + 1; c < U && c < Nc; ++c) BQ += fabs((double)Jb[a * ld + c]);
      const double R = 2.0 * Bv + 2.0 * BQ + 2.0 * margin + 1.0;
      const double room = 32768.0 - (U + 1) - U - 2.0;
      if (!isfinite(R)) return 0.0f;
      int e = (int)floor(log2(room / R)) + 1;
      while (ldexp(R, e) > room) --e;
      return e >= -100 ? (float)ldexp(1.0, e) : 0.0f;
    };
    P->pk_scale = pk_scale_of(kUWide);
    P->pk_slack = kUWide + 1;
    P->pk_scale10 = pk10 ? pk_scale_of(kUPk) : 0.0f;
    P->pk_slack10 = kUPk + 1;
    // Three-field walk: a field's value is u = (G - fastThr) sc - (U + 1)
    // relative to its test bit, plus rounding, and a block moves it by at
    // most Rb = sum_f |x_f| units, x_f = rint(WL_f sc) + rint(Wrec_f sc) the
    // packed step of low spin f.  The walk clamps every start to
    // [Rb - kTriRoom, kTriRoom - 1 - Rb] (re-walking the block when it lay
    // below), so no field leaves its range while Rb <= (kTriRoom - 1) / 2.
    // Rb = (lane part: sum_f |rint(WL_f sc)|, summed by the walk) + pk_rb3,
    // with pk_rb3 >= sc Rrec + U / 2 and Rrec = sum_{f<U} 2 (|h_f| +
    // sum_{U <= g < min(N, kMaxFree)} |J_fg|) >= sum_f |Wrec_f| for every
    // block.  sc: the largest power of two for which Rrec plus 1.5 times the
    // RMS size of the lane part (prefix spins from kUPk + kTriMinM up) stays
    // inside that room -- lanes whose lane part exceeds it re-walk every
    // block -- and at most 2^7 times the paired scale (so that every value
    // of the start computation is exact in fp32).
    float sc3 = 0.0f;
    int rb3 = 0;
    if (pk10 && P->pk_scale10 > 0.0f) {
      double rrec = 0.0, lrms = 0.0;
      for (int f = 0; f < kUPk && f < Nc; ++f) {
        double a = fabs((double)hb[f]), q = 0.0;
        for (int g = kUPk; g < Nc; ++g) {
          const double j = (double)(f < g ? Jb[f * ld + g] : Jb[g * ld + f]);
          if (g < kMaxFree) a += fabs(j);
          if (g >= kUPk + kTriMinM) q += j * j;
        }
        rrec += 2.0 * a;
        lrms += 2.0 * sqrt(q);
      }
      const double room = 0.5 * (kTriRoom - 1) - 0.5 * kUPk - 2.0;
      const double need = (rrec + 1.5 * lrms) * (1.0 + 1.0 / 1024.0);
      double s3 = 128.0 * (double)P->pk_scale10;
      while (s3 * need > room && s3 > 1e-30) s3 *= 0.5;
      sc3 = (float)s3;
      rb3 = (int)ceil(s3 * rrec * (1.0 + 1.0 / 1024.0) + 0.5 * kUPk) + 1;
    }
    P->pk_scale3 = sc3;
    P->pk_rb3 = rb3;
    P->thr_key = 0xFFFFFFFFu;
    P->rec_count = 0;
    P->thr_mask = ~0ull;
    P->margin = (float)margin;
    P->qmin_f[0] = f32_down(qmin7);
    P->qmin_i[0] = (int32_t)qmin7;
    P->qmin_f[1] = f32_down(qmin8);
    P->qmin_i[1] = (int32_t)qmin8;
    P->qmin_f[2] = f32_down(qmin10);
    P->qmin_i[2] = (int32_t)qmin10;
    P->err = err;
    P->cand_count = 0;
    P->surv_count = 0;
    P->redo = 0;
    P->walk_f32 = walk_f32 ? 1u : 0u;
    P->stat_redo = 0;
    P->bound = Bv;
    P->stat_candidates = 0;
    P->stat_slow = 0;
    P->max_drift_bits = 0;
    P->max_chunk_cand = 0;
  }
}

// ---------------------------------------------------------------- k_tables
// Record of block T for n free spins (spins 0..n-1; low = 0..U-1,
// high = U..n-1), free configuration x = gray(T << U) at the block start:
//   w[0] cB(T)  = 2 sigma_g (h_g + sum_{j<n, j!=g} J_gj s_j), the uniform
//                 part of the energy change when the boundary step flips the
//                 high spin g = U + ctz(T) whose old value is sigma_g (T >= 1)
//   w[1] R(T)   = E_FF(x) - Q(x_low): energy of the free spins alone minus
//                 the low-low part (used by the fp32 re-anchor)
//   w[2+f]      = Wu_f(T) = 2 (h_f + sum_{g high} J_fg s_g) for low f < U-1,
//                 and sigma_T Wu_{U-1}(T) for f = U-1 with sigma_T = +1 for
//                 odd T, -1 for even T (old value of spin U-1 when the inner
//                 step 2^(U-1) flips it).
// Tables for n = U .. nmax are concatenated; the table of n starts at record
// 2^(n-U) - 1.  grid.y indexes the instance.  The search uses U = kU or
// kUWide (words of kRecWords) and kUPk (single searches, rec_words(kUPk)
// words); the log Z walk (kF64) U = kLzU or kLzUF and records of 2 + U
// doubles.

template <bool kInt, bool kF64, int U>
__global__ void k_tables(Batch bt, int ncap, void* out, int paired) {
  static_assert(kF64 || 2 + U <= rec_words(U), "record exceeds its words");
  const int b = blockIdx.y;
  const int N = inst_N(bt, b);
  if (N < U || N > bt.ld) return;
  const int nmax = min(ncap, N);
  const int64_t total = ((int64_t)1 << (nmax - U + 1)) - 1;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= total) return;
  // which n: records of n occupy [2^(n-U) - 1, 2^(n-U+1) - 1)
  int n = U;
  while (((int64_t)1 << (n - U + 1)) - 1 <= r) ++n;
  const uint32_t T = (uint32_t)(r - (((int64_t)1 << (n - U)) - 1));
  const int ld = bt.ld;
  const uint32_t x = gray32(T << U);
  using Tv = typename std::conditional<kInt, int32_t, float>::type;
  const Tv* Jb = inst_J<Tv>(bt, b);
  const Tv* hb = inst_h<Tv>(bt, b);
  auto J = [&](int a, int c) -> double { return (double)(a < c ? Jb[a * ld + c] : Jb[c * ld + a]); };
  auto H = [&](int a) -> double { return (double)hb[a]; };
  auto S = [&](int j) -> double { return ((x >> j) & 1u) ? 1.0 : -1.0; };

  double cB = 0.0;
  if (T >= 1) {
    const int c = __builtin_ctz(T);
    const int g = U + c;
    const double sig = ((T >> (c + 1)) & 1u) ? 1.0 : -1.0;
    double fld = H(g);
    for (int j = 0; j < n; ++j)
      if (j != g) fld += J(g, j) * S(j);
    cB = 2.0 * sig * fld;
  }
  double eff = 0.0;
  for (int a = 0; a < n; ++a) {
    double f = H(a);
    for (int c = a + 1; c < n; ++c) f += J(a, c) * S(c);
    eff -= S(a) * f;
  }
  double q = 0.0;
  for (int a = 0; a < U; ++a)
    for (int c = a + 1; c < U; ++c) q -= J(a, c) * S(a) * S(c);
  const double R = eff - q;
  // Wu_f of the block whose free configuration is xb (parity of T)
  auto wu_of = [&](uint32_t xb, double* w) {
    for (int f = 0; f < U; ++f) {
      double s = H(f);
      for (int g = U; g < n; ++g) s += J(f, g) * (((xb >> g) & 1u) ? 1.0 : -1.0);
      w[f] = 2.0 * s;
    }
    w[U - 1] *= (T & 1u) ? 1.0 : -1.0;
  };
  double wu[U];
  wu_of(x, wu);

  if (kF64) {  // records of 2 + U doubles (the log Z walk keeps its energies in fp64)
    double* rec = (double*)out + ((size_t)b * bt.table_recs + (size_t)r) * (2 + U);
    rec[0] = cB;
    rec[1] = R;
    for (int f = 0; f < U; ++f) rec[2 + f] = wu[f];
    return;
  }
  // search tables of U = kUWide follow those of U = kU at record table_base8;
  // those of U = kUPk (records of rec_words(kUPk)) start at word table_base10w
  uint32_t* rec;
  if (U == kUPk) {
    rec = bt.table + (size_t)b * bt.table_recs * kRecWords + (size_t)bt.table_base10w +
          (size_t)r * rec_words(U);
  } else {
    const int64_t base = U == kUWide ? bt.table_base8 : 0;
    rec = bt.table + ((size_t)b * bt.table_recs + (size_t)(base + r)) * kRecWords;
  }
  if (kInt && !bt.P[b].walk_f32) {
    rec[0] = (uint32_t)(int32_t)cB;
    rec[1] = (uint32_t)(int32_t)R;
    for (int f = 0; f < U; ++f) rec[2 + f] = (uint32_t)(int32_t)wu[f];
  } else {
    rec[0] = __float_as_uint((float)cB);
    rec[1] = __float_as_uint((float)R);
    for (int f = 0; f < U; ++f) rec[2 + f] = __float_as_uint((float)wu[f]);
    // packed steps of the three-field walk: the record of block T of the
    // first stream of a level (T - b < Q) holds those of the triple
    // (T, T + Q, T + 2Q), all three of the parity of T, after the paired
    // walk's (both are written: the host picks the walk per chunk)
    const float s3 = U == kUPk ? bt.P[b].pk_scale3 : 0.0f;
    const bool tri = paired && U == kUPk && bt.tri && n >= U + kTriMinM && s3 > 0.0f;
    if (tri) {
      uint32_t base = 0, Q = 1u << (n - U - 2);
      while (Q >= 2u && T >= base + 3u * Q) {
        base += 3u * Q;
        Q >>= 2;
      }
      if (Q >= 2u && T < base + Q) {
        double wb[U], wc[U];
        wu_of(gray32((T + Q) << U), wb);
        wu_of(gray32((T + 2u * Q) << U), wc);
        for (int f = 0; f < U; ++f) {
          const uint32_t xa = (uint32_t)(int32_t)rintf((float)wu[f] * s3);
          const uint32_t xb = (uint32_t)(int32_t)rintf((float)wb[f] * s3);
          const uint32_t xc = (uint32_t)(int32_t)rintf((float)wc[f] * s3);
          rec[kPkWordTri + f] = xa + (xb << kTriShiftB) + (xc << kTriShiftC);
        }
      }
    }
    // packed steps of the paired walk: blocks T and T ^ half (same parity)
    const float sc = U == kUPk ? bt.P[b].pk_scale10 : bt.P[b].pk_scale;
    if (paired && (U == kUWide || U == kUPk) && n >= U + 2 && sc > 0.0f) {
      const uint32_t half = 1u << (n - U - 1);
      const uint32_t T2 = T ^ half;
      double wp[U];
      wu_of(gray32(T2 << U), wp);
      const bool first = T < half;  // this record is block A of its pair
      constexpr int kIn = pk_in_a(U);
      for (int f = first ? 0 : kIn; f < (first ? kIn : U); ++f) {
        const int32_t xs = (int32_t)rintf((float)wu[f] * sc);
        const int32_t xp = (int32_t)rintf((float)wp[f] * sc);
        const uint32_t xa = (uint32_t)(first ? xs : xp), xb = (uint32_t)(first ? xp : xs);
        rec[pk_word(U) + (first ? f : f - kIn)] = xa + (xb << 16);
      }
    }
  }
}

// ------------------------------------------------------------------ k_enum
// One lane per prefix p (spins n..N-1 fixed to the bits of p); the lane walks
// all 2^n configurations of the free spins in reflected Gray-code order,
// blocks of 2^U steps at a time.  Every state costs one add (its G, the
// energy minus the low-low part) and one order test against the bound
// fastThr = threshold - (smallest low-low energy), which no state below the
// threshold can exceed.  Two walks:
//   plain  -- G in fp32 (or int32); the block minimum, one 3-input min per
//             two states, against the bound;
//   paired -- (fp32 walks; blocks of 8 with n >= 10, and in single
//             searches blocks of 10 with n >= 12) blocks T
//             and T + 2^(n-U-1) in the two 16-bit fixed-point fields of one
//             word: one integer add and one AND per step for both states,
//             the sign bit of each field the test.
// A block that may hold a state below the bound is walked again in fp32 (or
// int32), each state tested exactly, and every state at or below the
// threshold is appended as a candidate mask.  blockIdx.x / blocks_per_inst
// selects the instance.

template <typename V>
struct Num;
template <>
struct Num<float> {
  static __device__ inline float mn(float a, float b) { return fminf(a, b); }
  static __device__ inline float big() { return __int_as_float(0x7f800000); }
};
template <>
struct Num<int32_t> {
  static __device__ inline int32_t mn(int32_t a, int32_t b) { return min(a, b); }
  static __device__ inline int32_t big() { return 1 << 29; }
};

template <bool kInt, bool kWF, int U, bool kSplit, bool kPk, bool kTri = false>
__device__ __forceinline__ void enum_walk(const Batch& bt, const void* __restrict__ Jv,
                                          const void* __restrict__ hv,
                                          const uint32_t* __restrict__ table,
                                          const uint32_t* __restrict__ qtab_all, const Chunk& ch,
                                          int b, int blk, int N, int n, int64_t lanes, Params* P,
                                          uint32_t* s_yw, void* s_Fw, void* s_Rw, void* s_EHw);

// U: low spins per block (kU, kUWide or kUPk; n >= U for every chunk).  kSplit: the
// bound is tested per sub-block of 64 steps instead of per block (batches,
// whose short levels bring many candidates per state).
// Resident waves: 8 per SIMD (64 VGPRs); the walk over blocks of kUPk
// carries ten packed steps and three group steps and takes 7 (72 VGPRs,
// 4825 ms per N = 48 search against 4929 ms at 8 waves, where it spills its
// per-block values).  kTri: the three-field walk (blocks of kUPk, single
// searches, n >= kUPk + kTriMinM).
template <bool kInt, int U, bool kSplit, bool kPk, bool kTri = false>
__global__ __launch_bounds__(kEnumBlock, U == kUPk ? 7 : 8) void k_enum(Batch bt, const void* __restrict__ Jv,
                                                        const void* __restrict__ hv,
                                                        const uint32_t* __restrict__ table,
                                                        const uint32_t* __restrict__ qtab_all,
                                                        Chunk ch, int blocks_per_inst) {
  using A = typename std::conditional<kInt, int64_t, double>::type;  // exact init

  const int b = blockIdx.x / blocks_per_inst;
  const int blk = blockIdx.x - b * blocks_per_inst;
  const int N = inst_N(bt, b);
  const int n = ch.n;
  // this chunk's masks must lie inside the instance's state space
  if (N < n || N > bt.ld || (N < 63 && ch.first_mask >= (1ull << N))) return;
  const int64_t lanes = N < 63 ? min(ch.lanes, (int64_t)(((1ull << N) - ch.first_mask) >> n))
                               : ch.lanes;
  Params* P = bt.P + b;
  const uint32_t err0 = P->err;
  if (err0 & (kErrNonFinite | kErrOverflow | kErrInval)) return;
  if (ch.retry && !P->redo) return;

  // LDS shared by both walk variants: the lane's high-spin fields Y_g (index
  // [g - U][thread], read once per block boundary), which first hold the
  // staged couplings, and the workgroup's sums over its upper prefix spins.
  __shared__ uint32_t s_y[kMaxHigh * kEnumBlock];
  __shared__ A s_F[2][kMaxFree + 8];
  __shared__ A s_R[2][kMaxN];
  __shared__ A s_EH[2];
  if constexpr (U == kUPk) {
    // blocks of 10: fp32 walks; an integer instance that takes the int32
    // walk walks the chunk's blocks of 8 instead
    if (!kInt || P->walk_f32) {
      enum_walk<kInt, true, kUPk, kSplit, true, kTri>(bt, Jv, hv, table, qtab_all, ch, b, blk,
                                                      N, n, lanes, P, s_y, s_F, s_R, s_EH);
    } else if constexpr (kInt) {
      Chunk c8 = ch;
      c8.table_offset = ch.table_offset8;
      enum_walk<true, false, kUWide, kSplit, false>(bt, Jv, hv, table, qtab_all, c8, b, blk, N,
                                                    n, lanes, P, s_y, s_F, s_R, s_EH);
    }
  } else {
    if (kInt && P->walk_f32)
      enum_walk<true, true, U, kSplit, kPk>(bt, Jv, hv, table, qtab_all, ch, b, blk, N, n,
                                            lanes, P, s_y, s_F, s_R, s_EH);
    else
      enum_walk<kInt, !kInt, U, kSplit, kPk && !kInt>(bt, Jv, hv, table, qtab_all, ch, b, blk, N,
                                                      n, lanes, P, s_y, s_F, s_R, s_EH);
  }
}

// The walk of k_enum.  kInt: the instance is int32 (exact set-up in int64,
// integer keys); kWF: the walk runs in fp32 (fp32 instances, and integer ones
// whose values fit 24 bits, whose tables then hold fp32 values).
template <bool kInt, bool kWF, int U, bool kSplit, bool kPk, bool kTri>
__device__ __forceinline__ void enum_walk(const Batch& bt, const void* __restrict__ Jv,
                                          const void* __restrict__ hv,
                                          const uint32_t* __restrict__ table,
                                          const uint32_t* __restrict__ qtab_all, const Chunk& ch,
                                          int b, int blk, int N, int n, int64_t lanes, Params* P,
                                          uint32_t* s_yw, void* s_Fw, void* s_Rw, void* s_EHw) {
  using V = typename std::conditional<kWF, float, int32_t>::type;
  using A = typename std::conditional<kInt, int64_t, double>::type;  // exact init
  using Ts = typename std::conditional<kInt, int32_t, float>::type;  // stored values
  static_assert(U >= kU, "s_y holds the kMaxFree - kU high fields of the smallest blocks");
  constexpr int kSteps = 1 << U;                            // steps per block
  constexpr int kReBlocks = 1 << (kReanchorLog2 - U);       // fp32: blocks per re-anchor
  V* s_y = (V*)s_yw;
  const uint32_t* qtab = qtab_all + (size_t)b * kQStride + qtab_base(U);  // uniform: SGPRs
  constexpr int kQi = qmin_index(U);  // this block size's Q minimum
  constexpr int kRW = rec_words(U);   // words per table record

  const int tid = threadIdx.x;
  const int ld = bt.ld;
  const int64_t lane = (int64_t)blk * kEnumBlock + tid;
  const bool valid = lane < lanes;
  // the workgroup's lanes hold the consecutive prefixes p0 .. p0 + 255
  const uint64_t p0 = ch.prefix_base + (uint64_t)blk * kEnumBlock;
  const uint64_t p = p0 + (uint64_t)(valid ? tid : 0);
  const uint32_t* tab =
      U == kUPk ? table + (size_t)b * bt.table_recs * kRecWords + (size_t)bt.table_base10w +
                      (size_t)ch.table_offset * kRW
                : table + ((size_t)b * bt.table_recs + (size_t)ch.table_offset) * kRecWords;
  uint64_t* cand = bt.cand + (size_t)b * bt.cap;
  uint32_t* ckey = bt.ckey + (size_t)b * bt.cap;
  const uint32_t cand_cap = bt.cap;

  const Ts* Jt = (const Ts*)Jv + (size_t)b * ld * ld;
  const Ts* ht = (const Ts*)hv + (size_t)b * ld;

  // ---- per-lane init (exact in int64 / fp64) --------------------------------
  // y_f = sum_{q >= n} J_fq s_q (field on free spin f from the prefix);
  // E_P = energy of the prefix spins alone.  WL_f = 2 y_f for the low spins,
  // Y_g = 2 y_g for the high ones.
  // The prefix spins split into the kLaneBits lowest ("L": spins n .. n+kl-1,
  // different in every lane) and the rest ("H": spins n+kl .. N-1, bits of
  // p >> kLaneBits, which is h0 or h0 + 1 in a workgroup).  The H parts --
  // the fields F of H on the free and L spins and the energy E_H of H alone --
  // are summed once per workgroup for both values of p >> kLaneBits; a lane
  // adds only the kl L spins on top.  Every coupling read here has its
  // column among the prefix spins, so the stage holds columns n .. N-1 of J
  // (row stride kp = N - n) and the prefix spins' fields: N kp + kp <= 63 x 56
  // + 56 values, which fit in the space of the high fields (written only once
  // the stage has been read).
  constexpr int kLaneBits = 8;  // log2(kEnumBlock)
  const int kl = min(N - n, kLaneBits);
  const int qh = n + kl;      // first H spin
  const int nf = n + kl;      // spins that take a field from H
  const uint64_t h0 = p0 >> kLaneBits;
  A(*s_F)[kMaxFree + kLaneBits] = (A(*)[kMaxFree + kLaneBits])s_Fw;
  A(*s_R)[kMaxN] = (A(*)[kMaxN])s_Rw;
  A* s_EH = (A*)s_EHw;
  const int kp = N - n;
  static_assert(kMaxN * (kMaxN - U) + (kMaxN - U) <= kMaxHigh * kEnumBlock,
                "coupling stage exceeds s_y");
  V* s_stage = s_y;  // s_stage[i kp + q - n] = J_iq (q >= n); then h_q at N kp + q - n
  const V* s_hp = s_stage + N * kp;
  for (int k = tid; k < N * kp + kp; k += kEnumBlock)
    s_stage[k] = k < N * kp ? (V)Jt[(k / kp) * ld + n + (k % kp)] : (V)ht[n + k - N * kp];
  __syncthreads();
  for (int t = tid; t < 2 * nf; t += kEnumBlock) {
    const int c = t >= nf, i = t - c * nf;
    const uint64_t hb = h0 + (uint64_t)c;
    A acc = 0;
    for (int q = qh; q < N; ++q) {
      const A jq = (A)s_stage[i * kp + q - n];
      acc += ((hb >> (q - qh)) & 1ull) ? jq : -jq;
    }
    s_F[c][i] = acc;
  }
  for (int t = tid; t < 2 * (N - qh); t += kEnumBlock) {
    const int c = t >= N - qh, q = qh + t - c * (N - qh);
    const uint64_t hb = h0 + (uint64_t)c;
    A f = (A)s_hp[q - n];
    for (int r = q + 1; r < N; ++r) {
      const A jr = (A)s_stage[q * kp + r - n];
      f += ((hb >> (r - qh)) & 1ull) ? jr : -jr;
    }
    s_R[c][q - qh] = ((hb >> (q - qh)) & 1ull) ? f : -f;
  }
  __syncthreads();
  if (tid < 2) {
    A e = 0;
    for (int q = 0; q < N - qh; ++q) e -= s_R[tid][q];
    s_EH[tid] = e;
  }
  __syncthreads();
  const int c = (int)((p >> kLaneBits) - h0);  // 0 or 1
  const uint32_t plo = (uint32_t)p;            // bit j: spin n + j (j < kl)
  V WL[U];
  A ysum = 0;
#pragma unroll
  for (int f = 0; f < U; ++f) {
    A acc = s_F[c][f];
    for (int j = 0; j < kl; ++j) {
      const A jq = (A)s_stage[f * kp + j];
      acc += ((plo >> j) & 1u) ? jq : -jq;
    }
    ysum += acc;
    WL[f] = valid ? (V)(2 * acc) : (V)0;
  }
  V yh[kMaxHigh];
#pragma unroll
  for (int k = 0; k < kMaxHigh; ++k) {
    yh[k] = (V)0;
    if (k < n - U) {
      A acc = s_F[c][U + k];
      for (int j = 0; j < kl; ++j) {
        const A jq = (A)s_stage[(U + k) * kp + j];
        acc += ((plo >> j) & 1u) ? jq : -jq;
      }
      ysum += acc;
      yh[k] = valid ? (V)(2 * acc) : (V)0;
    }
  }
  A EP = s_EH[c];
  for (int j = 0; j < kl; ++j) {
    const int q = n + j;
    A f = (A)s_hp[j] + s_F[c][q];
    for (int r = j + 1; r < kl; ++r) {
      const A jr = (A)s_stage[q * kp + r];
      f += ((plo >> r) & 1u) ? jr : -jr;
    }
    EP -= ((plo >> j) & 1u) ? f : -f;
  }
  __syncthreads();  // every lane has read the stage
#pragma unroll
  for (int k = 0; k < kMaxHigh; ++k)
    if (k < n - U) s_y[k * kEnumBlock + tid] = yh[k];
  V G;
  {
    const uint32_t r0 = tab[1];
    const A R0 = kWF ? (A)__uint_as_float(r0) : (A)(int32_t)r0;
    G = valid ? (V)(EP + ysum + R0) : Num<V>::big();
  }
  // fp32 re-anchor constants: E_P minus the low spins' prefix fields at a
  // block start of either parity (low spins all -1, except spin U-1 = +1 in
  // odd blocks), from the rounded fields the walk itself uses.
  float epa0 = 0.0f, epa1 = 0.0f;
  if (kWF) {
    double lo = 0.0;
    for (int f = 0; f < U - 1; ++f) lo += 0.5 * (double)WL[f];
    const double yl = 0.5 * (double)WL[U - 1];
    epa0 = (float)((double)EP + lo + yl);
    epa1 = (float)((double)EP + lo - yl);
  }
  __syncthreads();  // s_y visible

  // ---- thresholds ------------------------------------------------------------
  const uint32_t thr_key = P->thr_key;
  const uint64_t thr_mask = P->thr_mask;
  const bool full = P->rec_count != 0 && thr_key != 0xFFFFFFFFu;
  V thrE, fastThr;
  if (kInt) {
    int64_t t = full ? (int64_t)i32_of_key(thr_key) : (int64_t)(1 << 29);
    // chunks ascend in mask order: once the record is full every state here
    // has a larger mask than the S-th entry, so a tie with it cannot enter
    if (full && ch.first_mask > thr_mask) t -= 1;
    thrE = (V)t;
    fastThr = (V)(t - (int64_t)P->qmin_i[kQi]);
  } else {
    if (full) {
      const float tk = __uint_as_float(bits_of_f32_key(thr_key));
      float te;
      if (P->margin > 0.0f) {
        te = f32_up((double)tk + (double)P->margin);
      } else {
        // exact fp32 instance: the integer tie rule applies unchanged
        te = (ch.first_mask > thr_mask) ? nextafterf(tk, -__int_as_float(0x7f800000)) : tk;
      }
      thrE = (V)te;
      fastThr = (V)f32_up((double)te - (double)P->qmin_f[kQi]);
    } else {
      thrE = Num<V>::big();
      fastThr = Num<V>::big();
    }
  }

  const uint32_t nblocks = 1u << (n - U);
  float drift = 0.0f;
  uint32_t slow = 0;  // wave-blocks that took the re-walk (wave-uniform)

  // With kSplit the minimum is kept per sub-block of 64 steps, and G at every
  // sub-block start, so that a block whose bound passes re-walks only the
  // sub-blocks that can hold a state below the threshold (a few more
  // instructions per block, far fewer re-walked states where candidates are
  // frequent); without it the block is one sub-block.
  constexpr int kSub = kSplit ? 64 : kSteps;
  constexpr int kNSub = kSteps / kSub;
  constexpr int kHitWords = kSteps / 64;  // hit masks: one bit per state
  static_assert(kSteps % kSub == 0 && kSub % 64 == 0, "sub-blocks of whole hit words");

  // Re-walk of block T (steps W, sub-block start values gsub), testing every
  // state exactly, of the sub-blocks whose `pass` bit is set in some lane;
  // the states at or below thrE in lanes that passed become candidates.
  auto rewalk = [&](uint32_t T, const V (&W)[U], const V (&gsub)[kNSub],
                    const bool (&pass)[kNSub]) {
   if constexpr (kSteps <= 256) {
    ++slow;
    const uint32_t* q = qtab + (T & 1u) * kSteps;
    const V Gs = gsub[0];
    uint64_t hits[kHitWords];
#pragma unroll
    for (int k = 0; k < kHitWords; ++k) hits[k] = 0ull;
    auto qv = [&](int i) -> V { return kWF ? (V)__uint_as_float(q[i]) : (V)(int32_t)q[i]; };
#pragma unroll
    for (int w = 0; w < kNSub; ++w) {
      if (kSplit && __ballot(pass[w]) == 0ull) continue;  // wave-uniform
      // the opaque copy keeps the compiler from holding the values of the
      // fast walk live across the branch
      V g2 = gsub[w];
      asm volatile("" : "+v"(g2));
      if (g2 + qv(kSub * w) <= thrE) hits[(kSub * w) >> 6] |= 1ull;
#pragma unroll
      for (int j = 1; j < kSub; ++j) {
        const int i = kSub * w + j;
        const int f = __builtin_ctz(i);
        if (f == U - 1) g2 = g2 + W[f];
        else g2 = ((i >> (f + 1)) & 1) ? g2 + W[f] : g2 - W[f];
        if (g2 + qv(i) <= thrE) hits[i >> 6] |= (1ull << (i & 63));
      }
      if (!(valid && pass[w])) {
#pragma unroll
        for (int k = 0; k < kSub / 64; ++k) hits[(kSub * w) / 64 + k] = 0ull;
      }
    }
    // one slot reservation for all hits of the wave: an exclusive scan of
    // the lanes' hit counts, one atomic, then every lane writes its own
    // hits from its offset (the atomic's latency is paid once per block,
    // not once per step that hits)
    uint32_t nh = 0;
#pragma unroll
    for (int w = 0; w < kHitWords; ++w) nh += (uint32_t)__popcll(hits[w]);
    uint32_t incl = nh;
#pragma unroll
    for (int o = 1; o < kWaveLanes; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if ((int)__lane_id() >= o) incl += y;
    }
    const uint32_t total = __shfl(incl, kWaveLanes - 1);
    uint32_t base = 0;
    if (__lane_id() == 0 && total != 0) base = atomicAdd(&P->cand_count, total);
    uint32_t slot = __shfl(base, 0) + incl - nh;
    const uint64_t pl = ch.prefix_base + (uint64_t)lane;
#pragma unroll
    for (int w = 0; w < kHitWords; ++w) {
      uint64_t hw = hits[w];
      while (hw) {
        const int i = 64 * w + __builtin_ctzll(hw);
        hw &= hw - 1ull;
        const uint64_t t = ((uint64_t)T << U) | (uint64_t)i;
        const uint64_t mask = (pl << n) | (t ^ (t >> 1));
        // the walk's energy of step i, from the block start: a low spin
        // f < U-1 that is up at step i flipped an odd number of times from
        // -1 (net -W_f); spin U-1 flips once, at step 2^(U-1) (net +W_{U-1})
        const uint32_t gi = (uint32_t)(i ^ (i >> 1));
        V e = Gs;
#pragma unroll
        for (int f = 0; f < U - 1; ++f)
          if ((gi >> f) & 1u) e = e - W[f];
        if ((gi >> (U - 1)) & 1u) e = e + W[U - 1];
        e = e + qv(i);
        const uint32_t key = kInt ? key_of_i32((int32_t)e) : key_f32((float)e);
        // beyond cap the mask is dropped; the merge sees cand_count > cap
        // and asks for another pass over the chunk
        if (slot < cand_cap) {
          cand[slot] = mask;
          ckey[slot] = key;
        }
        ++slot;
      }
    }
   }
  };

  // Re-walk of a block of more than 256 steps (fp32 walks), as a loop over
  // its passes of 64 steps: pass w is walked when bit w of some lane's pmask
  // is set, from its start value (G0 and the net steps of the spins that are
  // up at step 64 w); its hits are appended at its end, with one slot
  // reservation per wave and pass that has any.
  auto rewalk_long = [&](uint32_t T, const V (&W)[U], V G0, uint32_t pmask) {
    ++slow;
    const uint32_t* q = qtab + (T & 1u) * kSteps;
    auto qv = [&](int i) -> V { return (V)__uint_as_float(q[i]); };
    const uint64_t pl = ch.prefix_base + (uint64_t)lane;
#pragma nounroll
    for (int w = 0; w < kSteps / 64; ++w) {
      const bool mine = (pmask >> w) & 1u;
      if (__ballot(mine) == 0ull) continue;  // wave-uniform
      const uint32_t g0 = (uint32_t)(64 * w) ^ (uint32_t)(32 * w);  // gray(64 w)
      V g2 = G0;
#pragma unroll
      for (int f = 5; f < U - 1; ++f)
        if ((g0 >> f) & 1u) g2 = g2 - W[f];
      if ((g0 >> (U - 1)) & 1u) g2 = g2 + W[U - 1];
      asm volatile("" : "+v"(g2));
      uint64_t hw = (g2 + qv(64 * w) <= thrE) ? 1ull : 0ull;
#pragma unroll
      for (int j = 1; j < 64; ++j) {
        const int f = __builtin_ctz(j);
        if (f == 5) g2 = (w & 1) ? g2 + W[5] : g2 - W[5];
        else g2 = ((j >> (f + 1)) & 1) ? g2 + W[f] : g2 - W[f];
        if (g2 + qv(64 * w + j) <= thrE) hw |= 1ull << j;
      }
      if (!mine) hw = 0ull;
      const uint32_t nh = (uint32_t)__popcll(hw);
      uint32_t incl = nh;
#pragma unroll
      for (int o = 1; o < kWaveLanes; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if ((int)__lane_id() >= o) incl += y;
      }
      const uint32_t total = __shfl(incl, kWaveLanes - 1);
      if (total == 0) continue;  // wave-uniform
      uint32_t base = 0;
      if (__lane_id() == 0) base = atomicAdd(&P->cand_count, total);
      uint32_t slot = __shfl(base, 0) + incl - nh;
      while (hw) {
        const int i = 64 * w + __builtin_ctzll(hw);
        hw &= hw - 1ull;
        const uint64_t t = ((uint64_t)T << U) | (uint64_t)i;
        const uint64_t mask = (pl << n) | (t ^ (t >> 1));
        const uint32_t gi = (uint32_t)(i ^ (i >> 1));
        V e = G0;
#pragma unroll
        for (int f = 0; f < U - 1; ++f)
          if ((gi >> f) & 1u) e = e - W[f];
        if ((gi >> (U - 1)) & 1u) e = e + W[U - 1];
        e = e + qv(i);
        const uint32_t key = key_f32((float)e);
        if (slot < cand_cap) {
          cand[slot] = mask;
          ckey[slot] = key;
        }
        ++slot;
      }
    }
  };

  // fresh G at the start of block T (fp32 walks): E_P minus the prefix fields
  // of the low spins (the parity constant), plus the record's R(T), minus the
  // high spins' prefix fields with their signs from the Gray code of T (one
  // LDS read and one fma per high spin)
  auto fresh_g = [&](uint32_t T, V RT) -> float {
    const uint32_t xh = gray32(T);  // high spins' bits
    float a = (float)(T & 1u ? epa1 : epa0) + (float)RT;
    for (int k = 0; k < n - U; ++k) {
      const float yg = (float)s_y[k * kEnumBlock + tid];
      a = fmaf(((xh >> k) & 1u) ? -0.5f : 0.5f, yg, a);
    }
    return a;
  };

  if constexpr (kPk && kTri) {
    static_assert(kWF && U == kUPk && !kSplit, "three-field walk: fp32, blocks of kUPk, searches");
    // ---- three-field walk -----------------------------------------------------
    // (chunks of a single search with n >= kUPk + kTriMinM.)  The blocks of a
    // triple (TA, TA + Q, TA + 2Q, all of the parity of TA) are walked as the
    // fields of one word: field k holds its bias plus u_k, u = (G - fastThr)
    // sc - (U + 1) plus at most U + 1 units of rounding, so its top bit
    // (bit 10, 21 or 31) is clear iff u < 0, which every state at or below
    // fastThr satisfies.  Steps, AND and the bound test are those of the
    // paired walk, on three blocks instead of two.  Each start u is clamped
    // to [Rb - kTriRoom, kTriRoom - 1 - Rb] (Rb: the lane's bound on a
    // block's summed step magnitudes), so that no field leaves its range; a
    // clamp from above hides no state below the bound (the block's states
    // all stay above the test bit), a clamp from below re-walks the block.
    const float sc = P->pk_scale3;
    const bool armed = full && sc > 0.0f;  // else every block is re-walked
    const float ftsc = armed ? fastThr * sc : 0.0f;  // exact: sc is a power of two
    // packed steps, carried from triple to triple as in the paired walk
    // (the triples of a lane alternate in parity, also across levels)
    uint32_t pk[U], rprev[U];
    int rbl = P->pk_rb3;
#pragma unroll
    for (int f = 0; f < U; ++f) {
      const int32_t xl = (int32_t)rintf((float)WL[f] * sc);
      pk[f] = (uint32_t)xl * kTriLane;
      rbl += xl < 0 ? -xl : xl;
      rprev[f] = 0u;
    }
    const bool lane_ok = 2 * rbl <= kTriRoom - 1;  // else the lane re-walks every block
    const float ulo = (float)(rbl - kTriRoom), uhi = (float)(kTriRoom - 1 - rbl);
    constexpr uint32_t kAll = (1u << (kSteps / 64)) - 1u;
    const int m = n - U;
    V GA = G, GB = G, GC = G;
    uint32_t base = 0;
#pragma nounroll
    for (uint32_t Q = 1u << (m - 2); Q >= 2u; Q >>= 2) {
      V ynext = s_y[tid];  // triple 1 flips high spin U in all three blocks
      for (uint32_t T = 0; T < Q; ++T) {
        const uint32_t TA = base + T, TB = TA + Q, TC = TB + Q;
        const uint32_t* recA = tab + (size_t)TA * kRW;
        const uint32_t* recB = tab + (size_t)TB * kRW;
        const uint32_t* recC = tab + (size_t)TC * kRW;
        auto rw = [&](const uint32_t* rec, int k) -> V { return (V)__uint_as_float(rec[k]); };
        uint32_t rpk[U];
#pragma unroll
        for (int f = 0; f < U; ++f) rpk[f] = recA[kPkWordTri + f];
        const V ycur = ynext;
        if (T + 1 < Q) ynext = s_y[__builtin_ctz(T + 1) * kEnumBlock + tid];
        const bool odd = T & 1u;
        if (T == 0) {
          // a level's blocks start from fresh values (block 0 from the lane's G)
          if (base != 0) GA = valid ? (V)fresh_g(TA, rw(recA, 1)) : G;
          GB = valid ? (V)fresh_g(TB, rw(recB, 1)) : G;
          GC = valid ? (V)fresh_g(TC, rw(recC, 1)) : G;
        } else {
          // boundary step of the three blocks: high spin U + c (base and Q
          // are multiples of 2^(c+1)), old value +1 iff bit c+1 of the
          // block's index is set
          const int c = __builtin_ctz(T);
          GA = ((TA >> (c + 1)) & 1u) ? GA + ycur : GA - ycur;
          GB = ((TB >> (c + 1)) & 1u) ? GB + ycur : GB - ycur;
          GC = ((TC >> (c + 1)) & 1u) ? GC + ycur : GC - ycur;
          GA = GA + rw(recA, 0);
          GB = GB + rw(recB, 0);
          GC = GC + rw(recC, 0);
          constexpr uint32_t kPkReBlocks = 1u << (kPkReanchorLog2 - U);
          if (!kInt && (T & (kPkReBlocks - 1)) == 0) {
            const float fa = valid ? fresh_g(TA, rw(recA, 1)) : (float)GA;
            const float fb = valid ? fresh_g(TB, rw(recB, 1)) : (float)GB;
            const float fc = valid ? fresh_g(TC, rw(recC, 1)) : (float)GC;
            drift = fmaxf(drift, fmaxf(fabsf((float)GA - fa),
                                       fmaxf(fabsf((float)GB - fb), fabsf((float)GC - fc))));
            GA = (V)fa;
            GB = (V)fb;
            GC = (V)fc;
          }
        }
        // clamped fixed-point starts (lanes past the chunk's end: any value
        // in range will do)
        auto ustart = [&](V Gx) -> float {
          return valid ? rintf(fmaf((float)Gx, sc, -ftsc)) - (float)(U + 1) : uhi;
        };
        const float xa = ustart(GA), xb = ustart(GB), xc = ustart(GC);
        const bool lowa = xa < ulo, lowb = xb < ulo, lowc = xc < ulo;
        auto field = [&](float x) -> uint32_t {
          return (uint32_t)(int32_t)fminf(fmaxf(x, ulo), uhi);
        };
        uint32_t g = field(xa) + (field(xb) << kTriShiftB) + (field(xc) << kTriShiftC) + kTriBias;
#pragma unroll
        for (int f = 0; f < U - 1; ++f) pk[f] = pk[f] + (rpk[f] - rprev[f]);
        // the lane's first triple is even: its top-spin lane part is minus
        // the lane's value
        pk[U - 1] = (base == 0 && T == 0) ? rpk[U - 1] - pk[U - 1]
                                          : (rpk[U - 1] + rprev[U - 1]) - pk[U - 1];
#pragma unroll
        for (int f = 0; f < U; ++f) rprev[f] = rpk[f];
        // sixteen 63-step passes in four groups of four, as in the paired walk
        uint32_t acc = 0xFFFFFFFFu;
        auto sub = [&](const uint32_t p5) {
          uint32_t accw = g;  // the pass's first state
#pragma unroll
          for (int j = 1; j < 64; ++j) {
            const int f = __builtin_ctz(j);
            if (f == 5) g = g + p5;
            else g = ((j >> (f + 1)) & 1) ? g + pk[f] : g - pk[f];
            asm volatile("v_and_b32 %0, %0, %1" : "+v"(accw) : "v"(g));
          }
          acc &= accw;
        };
        uint32_t p5 = 0u - pk[5];
        uint32_t s7 = 0u - pk[7];
        uint32_t t0 = 0u - pk[8] - pk[6], t1 = pk[U - 1] - pk[6], t2 = pk[8] - pk[6];
#pragma nounroll
        for (int o = 0; o < kSteps / 256; ++o) {
          uint32_t s0 = 0u - pk[6], s1 = s7, s2 = pk[6];
#pragma nounroll
          for (int w = 0; w < 4; ++w) {
            sub(p5);
            g = g + s0;
            s0 = s1;
            s1 = s2;
            p5 = 0u - p5;
          }
          g = g + t0;  // after the last group g is not used
          t0 = t1;
          t1 = t2;
          s7 = 0u - s7;
        }
        uint32_t ma = ((acc >> 10) & 1u) == 0u || lowa ? kAll : 0u;
        uint32_t mb = ((acc >> 21) & 1u) == 0u || lowb ? kAll : 0u;
        uint32_t mc = ((acc >> 31) & 1u) == 0u || lowc ? kAll : 0u;
        if (!armed || !lane_ok) ma = mb = mc = kAll;
        if (!valid) ma = mb = mc = 0u;
        const V wl = odd ? WL[U - 1] : -WL[U - 1];
        auto steps = [&](const uint32_t* rec, V (&W)[U]) {
#pragma unroll
          for (int f = 0; f < U - 1; ++f) W[f] = WL[f] + rw(rec, 2 + f);
          W[U - 1] = wl + rw(rec, 2 + U - 1);
        };
        if (__ballot(ma != 0u) != 0ull) {
          V W[U];
          steps(recA, W);
          rewalk_long(TA, W, GA, ma);
        }
        if (__ballot(mb != 0u) != 0ull) {
          V W[U];
          steps(recB, W);
          rewalk_long(TB, W, GB, mb);
        }
        if (__ballot(mc != 0u) != 0ull) {
          V W[U];
          steps(recC, W);
          rewalk_long(TC, W, GC, mc);
        }
        // the blocks end with spin U-1 up and every other low spin back down
        GA = GA + (wl + rw(recA, 2 + U - 1));
        GB = GB + (wl + rw(recB, 2 + U - 1));
        GC = GC + (wl + rw(recC, 2 + U - 1));
      }
      base += 3u * Q;
    }
    // the 2 or 4 blocks after the last level: walked exactly, from fresh values
    for (uint32_t T = base; T < nblocks; ++T) {
      const uint32_t* rec = tab + (size_t)T * kRW;
      V W[U];
#pragma unroll
      for (int f = 0; f < U - 1; ++f) W[f] = WL[f] + (V)__uint_as_float(rec[2 + f]);
      W[U - 1] = ((T & 1u) ? WL[U - 1] : -WL[U - 1]) + (V)__uint_as_float(rec[2 + U - 1]);
      const V G0 = valid ? (V)fresh_g(T, (V)__uint_as_float(rec[1])) : G;
      if (__ballot(valid) != 0ull) {
        rewalk_long(T, W, G0, valid ? kAll : 0u);
        --slow;  // not a block that the bound test sent back
      }
    }
  } else if constexpr (kPk) {
    static_assert(!kPk || (kWF && (U == kUWide || U == kUPk) && (!kSplit || kSub == 64)),
                  "paired walk: fp32 walks, blocks of 8 or 10, sub-blocks of 64");
    // ---- paired walk ----------------------------------------------------------
    // (blocks of kUWide, or of kUPk for the chunks of a single search with
    // n >= kUPk + 2.)  Blocks T and T + half (half = nblocks / 2, n >= U + 2:
    // both of the same parity) are walked together as the low and high 16-bit fields of one
    // 32-bit word, in fixed point with the power-of-two scale sc: a field
    // holds (G - fastThr) sc + 2^15 - slack, so that its bit 15 is clear iff
    // its state may lie below the bound.  Every Gray step is one integer add
    // of the packed step (W_f(T + half) sc << 16) + W_f(T) sc, exact as an
    // integer sum because no field leaves [0, 2^16) (range bounded in
    // k_prep), and one AND into an accumulator over both fields.  G itself is
    // carried in fp32 from block to block (boundary steps, the block's net
    // step +W_{U-1}, re-anchors) and turned into fixed point once per block.
    const uint32_t half = nblocks >> 1;
    const float sc = U == kUPk ? P->pk_scale10 : P->pk_scale;
    const uint32_t off = 32768u - (uint32_t)(U == kUPk ? P->pk_slack10 : P->pk_slack);
    const bool armed = full && sc > 0.0f;  // else every block is re-walked
    const float ftsc = armed ? fastThr * sc : 0.0f;  // exact: sc is a power of two
    // packed steps of the current pair: the lane's part (the same in both
    // fields) plus the records' part.  They are carried from pair to pair,
    // pk_f(T) = pk_f(T - 1) + (rpk_f(T) - rpk_f(T - 1)) with a wave-uniform
    // difference, and for the top spin, whose lane part changes sign with
    // the block parity, pk(T) = rpk(T) + rpk(T - 1) - pk(T - 1); so the lane
    // part is not kept in registers.
    uint32_t pk[U], rprev[U];
#pragma unroll
    for (int f = 0; f < U; ++f) {
      pk[f] = (uint32_t)(int32_t)rintf((float)WL[f] * sc) * 65537u;
      rprev[f] = 0u;
    }
    V GA = G, GB = G;
    V ynext = s_y[tid];  // pair 1 flips high spin U in both blocks
    for (uint32_t T = 0; T < half; ++T) {
      const uint32_t TB = T + half;
      const uint32_t* recA = tab + (size_t)T * kRW;
      const uint32_t* recB = tab + (size_t)TB * kRW;
      // record words are read where they are used (the re-walk reads its
      // steps itself), so that few of them stay live across the walk
      auto rw = [&](const uint32_t* rec, int k) -> V { return (V)__uint_as_float(rec[k]); };
      uint32_t rpk[U];
#pragma unroll
      for (int f = 0; f < U; ++f)
        rpk[f] = f < pk_in_a(U) ? recA[pk_word(U) + f] : recB[pk_word(U) + f - pk_in_a(U)];
      const V ycur = ynext;
      if (T + 1 < half) ynext = s_y[__builtin_ctz(T + 1) * kEnumBlock + tid];
      const bool odd = T & 1u;
      if (T == 0) {
        const float fb = fresh_g(TB, rw(recB, 1));
        GB = valid ? (V)fb : G;
      } else {
        // boundary step of both blocks: flip high spin U + c, old value +1
        // iff bit c+1 of the block index is set
        const int c = __builtin_ctz(T);
        GA = ((T >> (c + 1)) & 1u) ? GA + ycur : GA - ycur;
        GB = ((TB >> (c + 1)) & 1u) ? GB + ycur : GB - ycur;
        GA = GA + rw(recA, 0);
        GB = GB + rw(recB, 0);
        constexpr uint32_t kPkReBlocks = 1u << (kPkReanchorLog2 - U);
        if (!kInt && (T & (kPkReBlocks - 1)) == 0) {
          const float fa = valid ? fresh_g(T, rw(recA, 1)) : (float)GA;
          const float fb = valid ? fresh_g(TB, rw(recB, 1)) : (float)GB;
          drift = fmaxf(drift, fmaxf(fabsf((float)GA - fa), fabsf((float)GB - fb)));
          GA = (V)fa;
          GB = (V)fb;
        }
      }
      // fixed-point start values and packed steps
      // (lanes past the chunk's end hold no state: any finite value will do)
      const float ga = valid ? fmaf((float)GA, sc, -ftsc) : 0.0f;
      const float gb = valid ? fmaf((float)GB, sc, -ftsc) : 0.0f;
      const uint32_t za = (uint32_t)(int32_t)rintf(ga) + off;
      const uint32_t zb = (uint32_t)(int32_t)rintf(gb) + off;
#pragma unroll
      for (int f = 0; f < U - 1; ++f) pk[f] = pk[f] + (rpk[f] - rprev[f]);
      // block 0 is even: its top-spin lane part is minus the lane's value
      pk[U - 1] = T == 0 ? rpk[U - 1] - pk[U - 1] : (rpk[U - 1] + rprev[U - 1]) - pk[U - 1];
#pragma unroll
      for (int f = 0; f < U; ++f) rprev[f] = rpk[f];
      // Four sub-blocks of 64 steps in a loop.  Steps 64w + j, j = 1..63,
      // flip spin ctz(j) <= 5 with the sign of step j of sub-block 0, except
      // spin 5 (j = 32), whose sign alternates with w; step 64(w + 1) flips
      // spin 6 (down, then up) or 7.  (Unrolled over the whole block, the same
      // steps measured 43% of the VALU instructions issued in pairs against
      // 81% for the loop, and 18% slower.)
      // fired (batches): bit w (field A) / bit kFHi + w (field B) set when
      // sub-block w may hold a state below the bound
      constexpr int kFHi = kSteps / 64 <= 8 ? 8 : 16;
      uint32_t g = za + (zb << 16);
      uint32_t acc = 0xFFFFFFFFu;
      uint32_t fired = 0u;
      // one 63-step sub-block from state g (its first state already in g)
      auto sub = [&](const uint32_t p5, const int w) {
        uint32_t accw = g;  // state 64w
#pragma unroll
        for (int j = 1; j < 64; ++j) {
          const int f = __builtin_ctz(j);
          if (f == 5) g = g + p5;
          else g = ((j >> (f + 1)) & 1) ? g + pk[f] : g - pk[f];
          // the AND in walk order: left to the compiler, the chain of ANDs
          // is re-associated into a tree that keeps every step's value live
          asm volatile("v_and_b32 %0, %0, %1" : "+v"(accw) : "v"(g));
        }
        if (kSplit) {
          fired |= ((((accw >> 15) & 1u) ^ 1u) << w) | ((((accw >> 31) & 1u) ^ 1u) << (kFHi + w));
        } else {
          acc &= accw;
        }
      };
      // four passes, one per sub-block; spin 5 flips down in even sub-blocks
      // and up in odd ones, and the steps between them (64: spin 6 down,
      // 128: spin 7, 192: spin 6 up) rotate through three registers, so the
      // loop selects nothing.  (Unrolled into two passes of two sub-blocks,
      // the pairing fell from 86% to 72% and the search took 5% longer.)
      uint32_t p5 = 0u - pk[5];
      if constexpr (U == kUWide) {
        uint32_t s0 = 0u - pk[6], s1 = pk[U - 1], s2 = pk[6];
#pragma nounroll
        for (int w = 0; w < kSteps / 64; ++w) {
          sub(p5, w);
          g = g + s0;  // after the last sub-block g is not used
          s0 = s1;
          s1 = s2;
          p5 = 0u - p5;
        }
      } else {
        // blocks of 10: four groups of the same four passes.  Within a group
        // the steps between passes flip spin 6 (down), 7, 6 (up), spin 7 down
        // in even groups and up in odd ones; between groups spin 8 (down),
        // 9 (the block's top spin, up), 8 (up).  The group's last pass adds
        // spin 6's step once more, which the group step t takes back.
        uint32_t s7 = 0u - pk[7];
        uint32_t t0 = 0u - pk[8] - pk[6], t1 = pk[U - 1] - pk[6], t2 = pk[8] - pk[6];
#pragma nounroll
        for (int o = 0; o < kSteps / 256; ++o) {
          uint32_t s0 = 0u - pk[6], s1 = s7, s2 = pk[6];
#pragma nounroll
          for (int w = 0; w < 4; ++w) {
            sub(p5, 4 * o + w);
            g = g + s0;
            s0 = s1;
            s1 = s2;
            p5 = 0u - p5;
          }
          g = g + t0;  // after the last group g is not used
          t0 = t1;
          t1 = t2;
          s7 = 0u - s7;
        }
      }
      // which 64-step passes of each block to re-walk: bit w of ma / mb (every
      // pass of a block whose whole-block test fired, without kSplit)
      constexpr uint32_t kAll = (1u << (kSteps / 64)) - 1u;
      uint32_t ma, mb;
      if (kSplit) {
        ma = fired & kAll;
        mb = (fired >> kFHi) & kAll;
      } else {
        ma = (acc & 0x8000u) == 0u ? kAll : 0u;
        mb = (acc & 0x80000000u) == 0u ? kAll : 0u;
      }
      if (!armed) ma = mb = kAll;
      if (!valid) ma = mb = 0u;
      const bool anya = ma != 0u, anyb = mb != 0u;
      // per sub-block of the walk over blocks of 8 (one sub-block per block
      // without kSplit, one per pass with it)
      bool pa[kNSub], pb[kNSub];
#pragma unroll
      for (int w = 0; w < kNSub; ++w) {
        pa[w] = kSplit ? ((ma >> w) & 1u) != 0u : anya;
        pb[w] = kSplit ? ((mb >> w) & 1u) != 0u : anyb;
      }
      const V wl = odd ? WL[U - 1] : -WL[U - 1];
      // the fp32 steps of a block, formed only on the rare re-walk
      auto steps = [&](const uint32_t* rec, V (&W)[U]) {
#pragma unroll
        for (int f = 0; f < U - 1; ++f) W[f] = WL[f] + rw(rec, 2 + f);
        W[U - 1] = wl + rw(rec, 2 + U - 1);
      };
      // G at every sub-block start, from the block start: a low spin f < U-1
      // that is up at step i flipped an odd number of times from -1 (net
      // -W_f); spin U-1 flips once, at step 2^(U-1) (net +W_{U-1})
      auto starts = [&](V G0, const V (&W)[U], V (&gs)[kNSub]) {
#pragma unroll
        for (int w = 0; w < kNSub; ++w) {
          const uint32_t gi = gray32((uint32_t)(kSub * w));
          V e = G0;
#pragma unroll
          for (int f = 0; f < U - 1; ++f)
            if ((gi >> f) & 1u) e = e - W[f];
          if ((gi >> (U - 1)) & 1u) e = e + W[U - 1];
          gs[w] = e;
        }
      };
      if (__ballot(anya) != 0ull) {
        V W[U], gs[kNSub];
        steps(recA, W);
        if constexpr (kSteps > 256) {
          rewalk_long(T, W, GA, ma);
        } else {
          starts(GA, W, gs);
          rewalk(T, W, gs, pa);
        }
      }
      if (__ballot(anyb) != 0ull) {
        V W[U], gs[kNSub];
        steps(recB, W);
        if constexpr (kSteps > 256) {
          rewalk_long(TB, W, GB, mb);
        } else {
          starts(GB, W, gs);
          rewalk(TB, W, gs, pb);
        }
      }
      // the blocks end with spin U-1 up and every other low spin back down
      GA = GA + (wl + rw(recA, 2 + U - 1));
      GB = GB + (wl + rw(recB, 2 + U - 1));
    }
  } else {
    static_assert(U <= kUWide, "plain walk: blocks of at most 2^8 steps (unrolled)");
    V ynext = nblocks > 1 ? s_y[tid] : (V)0;  // block 1 flips high spin U

    for (uint32_t T = 0; T < nblocks; ++T) {
      const uint32_t* rec = tab + (size_t)T * kRecWords;
      V rw[2 + U];
#pragma unroll
      for (int k = 0; k < 2 + U; ++k)
        rw[k] = kWF ? (V)__uint_as_float(rec[k]) : (V)(int32_t)rec[k];
      const V ycur = ynext;
      if (T + 1 < nblocks) ynext = s_y[__builtin_ctz(T + 1) * kEnumBlock + tid];

      if (T != 0) {
        // boundary step: flip high spin g = U + c whose old value is +1 iff bit
        // c+1 of T is set
        const int c = __builtin_ctz(T);
        const bool up = (T >> (c + 1)) & 1u;
        G = up ? G + ycur : G - ycur;
        G = G + rw[0];
        if (!kInt && (T & (kReBlocks - 1)) == 0) {
          // fresh G = E_P - sum_f s_f y_f + R(T) in fp32 from the lane's fields
          const float fresh = valid ? fresh_g(T, rw[1]) : (float)G;
          drift = fmaxf(drift, fabsf((float)G - fresh));
          G = (V)fresh;
        }
      }

      V W[U];
#pragma unroll
      for (int f = 0; f < U - 1; ++f) W[f] = WL[f] + rw[2 + f];
      W[U - 1] = ((T & 1u) ? WL[U - 1] : -WL[U - 1]) + rw[2 + U - 1];

      // 2^U - 1 inner steps: one add per state, one 3-input min per two states
      V msub[kNSub], gsub[kNSub];
      gsub[0] = G;
      V m = G;
#pragma unroll
      for (int i = 1; i < kSteps; i += 2) {
        // odd step i flips spin 0; its old value is bit 1 of i
        G = ((i >> 1) & 1) ? G + W[0] : G - W[0];
        const V Ga = G;
        if (i + 1 < kSteps) {
          const int f = __builtin_ctz(i + 1);
          if (f == U - 1) G = G + W[f];
          else G = (((i + 1) >> (f + 1)) & 1) ? G + W[f] : G - W[f];
          if ((i + 1) % kSub == 0) {
            // step i closes sub-block (i + 1) / kSub - 1; step i + 1 opens the next
            msub[(i + 1) / kSub - 1] = Num<V>::mn(m, Ga);
            gsub[(i + 1) / kSub] = G;
            m = G;
          } else {
            m = Num<V>::mn(Num<V>::mn(m, Ga), G);
          }
        } else {
          msub[kNSub - 1] = Num<V>::mn(m, Ga);
        }
      }

      bool pass[kNSub];
      bool any = false;
#pragma unroll
      for (int w = 0; w < kNSub; ++w) {
        pass[w] = msub[w] <= fastThr;
        any = any || pass[w];
      }
      if (__ballot(any) != 0ull) rewalk(T, W, gsub, pass);
    }
  }

  // statistics: one atomic per wave
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) drift = fmaxf(drift, __shfl_xor(drift, o));
  if (__lane_id() == 0) {
    if (slow) atomicAdd(&P->stat_slow, (unsigned long long)slow);
    if (!kInt && drift > 0.0f) {
      atomicMax(&P->max_drift_bits, __float_as_uint(drift));
      // drift guard: the accumulated error must stay inside the margin
      if (drift > P->margin) atomicOr(&P->err, kErrDrift);
    }
  }
}

// Tiny instances (N < U): one thread per state, every state a candidate.
__global__ void k_direct(Batch bt, uint64_t lo, uint64_t hi) {
  const uint64_t m = lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= hi) return;
  Params* P = bt.P;
  const uint32_t slot = atomicAdd(&P->cand_count, 1u);
  if (slot < bt.cap) {
    bt.cand[slot] = m;
    bt.ckey[slot] = 0u;  // not used: the single search rescoring reads every candidate
  }
}

// ------------------------------------------------- scoring and merging
// Exact energy of each candidate (fp64 for float instances, rounded to fp32;
// int32 for integer ones); it survives if its key (E, mask) is below the S-th
// key of the record.

template <bool kInt>
__device__ inline uint32_t exact_key(const void* Js, const void* hs, int N, int ld, uint64_t m) {
  if (kInt) return key_of_i32(energy_i32((const int32_t*)Js, (const int32_t*)hs, N, ld, m));
  return key_f32((float)energy_f64((const float*)Js, (const float*)hs, N, ld, m));
}

// Stage instance b's J (N x N, stride N) and h into LDS.
template <bool kInt>
__device__ inline void stage_instance(const Batch& bt, int b, int N, uint32_t* s) {
  const uint32_t* Jb = (const uint32_t*)bt.J + (size_t)b * bt.ld * bt.ld;
  const uint32_t* hb = (const uint32_t*)bt.h + (size_t)b * bt.ld;
  for (int k = threadIdx.x; k < N * N + N; k += blockDim.x)
    s[k] = k < N * N ? Jb[(k / N) * bt.ld + (k % N)] : hb[k - N * N];
}

// Single instance: grid-stride over the candidates of instance b.
// In a repeated pass the record already holds some of the chunk's states:
// a candidate equal to a record entry is dropped.
__device__ inline bool in_record(const uint32_t* rkey, const uint64_t* rmask, uint32_t rn,
                                 uint32_t key, uint64_t m);

template <bool kInt>
__global__ void k_score(Batch bt, int b, int retry) {
  extern __shared__ uint32_t s_inst[];
  if (retry && !bt.P[b].redo) return;
  const int N = inst_N(bt, b);
  stage_instance<kInt>(bt, b, N, s_inst);
  __syncthreads();
  Params* P = bt.P + b;
  const uint64_t* cand = bt.cand + (size_t)b * bt.cap;
  uint32_t* skey = bt.skey + (size_t)b * bt.cap;
  uint64_t* smask = bt.smask + (size_t)b * bt.cap;
  const uint32_t cnt = min(P->cand_count, bt.cap);
  const uint32_t thr_key = P->thr_key;
  const uint64_t thr_mask = P->thr_mask;
  const bool full = P->rec_count != 0 && thr_key != 0xFFFFFFFFu;
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint32_t nround = (cnt + stride - 1) / stride;
  for (uint32_t r = 0; r < nround; ++r) {
    const uint32_t j = r * stride + blockIdx.x * blockDim.x + threadIdx.x;
    bool keep = false;
    uint64_t m = 0;
    uint32_t key = 0;
    if (j < cnt) {
      m = cand[j];
      key = exact_key<kInt>(s_inst, s_inst + N * N, N, N, m);
      keep = !full || key_less(key, m, thr_key, thr_mask);
      if (keep && retry)
        keep = !in_record(bt.rkey + (size_t)b * bt.S, bt.rmask + (size_t)b * bt.S,
                          P->rec_count, key, m);
    }
    if (keep) {
      const uint64_t act = __ballot(1);
      const int lid = __lane_id();
      const int leader = __ffsll((unsigned long long)act) - 1;
      uint32_t base = 0;
      if (lid == leader) base = atomicAdd(&P->surv_count, (uint32_t)__popcll(act));
      base = __shfl(base, leader);
      const uint32_t slot = base + (uint32_t)__popcll(act & ((1ull << lid) - 1ull));
      skey[slot] = key;
      smask[slot] = m;
    }
  }
}

__device__ inline void cmp_swap(uint32_t* k, uint64_t* m, uint32_t a, uint32_t b, bool asc) {
  const uint32_t ka = k[a], kb = k[b];
  const uint64_t ma = m[a], mb = m[b];
  const bool gt = key_less(kb, mb, ka, ma);  // a > b
  if (gt == asc) {
    k[a] = kb; k[b] = ka;
    m[a] = mb; m[b] = ma;
  }
}

__device__ inline void bitonic_sort(uint32_t* k, uint64_t* m, uint32_t P2) {
  for (uint32_t size = 2; size <= P2; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = threadIdx.x; t < P2 / 2; t += blockDim.x) {
        const uint32_t a = 2 * t - (t & (stride - 1));
        const uint32_t b = a + stride;
        const bool asc = (a & size) == 0;
        cmp_swap(k, m, a, b, asc);
      }
      __syncthreads();
    }
  }
}

// number of entries of sorted (k, m)[0..n) strictly less than (kx, mx)
__device__ inline uint32_t rank_in(const uint32_t* k, const uint64_t* m, uint32_t n, uint32_t kx,
                                   uint64_t mx) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (key_less(k[mid], m[mid], kx, mx)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ inline bool in_record(const uint32_t* rkey, const uint64_t* rmask, uint32_t rn,
                                 uint32_t key, uint64_t m) {
  const uint32_t r = rank_in(rkey, rmask, rn, key, m);
  return r < rn && rkey[r] == key && rmask[r] == m;
}

// k-th smallest (1-based) of keys[0..cnt) for the whole workgroup: four
// passes of 8-bit digits, most significant first, each a histogram in LDS and
// a scan of its 256 bins by the first 256 threads.  Needs blockDim.x a
// multiple of 256.
__device__ uint32_t radix_select(const uint32_t* keys, uint32_t cnt, uint32_t k, uint32_t* hist,
                                 uint32_t* state) {
  const uint32_t t = threadIdx.x;
  const bool bin = t < 256u;
  uint32_t prefix = 0u, pmask = 0u, rem = k;
  for (int shift = 24; shift >= 0; shift -= 8) {
    if (bin) hist[t] = 0u;
    __syncthreads();
    for (uint32_t j = t; j < cnt; j += blockDim.x) {
      const uint32_t key = keys[j];
      if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    // inclusive scan of the 256 bins (Hillis-Steele)
    uint32_t v = bin ? hist[t] : 0u;
    for (uint32_t o = 1; o < 256u; o <<= 1) {
      const uint32_t add = bin && t >= o ? hist[t - o] : 0u;
      __syncthreads();
      v += add;
      if (bin) hist[t] = v;
      __syncthreads();
    }
    const uint32_t before = t == 0 || !bin ? 0u : hist[t - 1];
    if (bin && before < rem && rem <= v) {
      state[0] = prefix | (t << shift);
      state[1] = rem - before;
    }
    __syncthreads();
    prefix = state[0];
    rem = state[1];
    pmask |= 255u << shift;
    __syncthreads();
  }
  return prefix;
}

// The whole workgroup: merge the ns survivors (skey, smask) with the sorted
// record, keeping the first S, and publish the S-th key as the threshold.
// Keys are distinct because masks are, so an entry's place is its rank among
// all of them.  Up to kRankByCount entries in all, the record and the
// survivors are put side by side in LDS and every rank is counted directly;
// beyond, the survivors are sorted (bitonic, in LDS when they fit, in global
// memory otherwise) and an element's rank is its index plus the number of
// smaller elements in the other list.  With `sel` (hist: 256 words, state:
// 3), more survivors than LDS holds are first cut to those at or below the
// S-th smallest survivor key: no other survivor can enter the record, since
// S survivors precede it.  They are sorted in LDS when they fit (ties at
// that key can exceed it; then all are sorted in global memory).
__device__ void merge_body(Params* P, int S, uint32_t cap, bool last_pass, uint32_t ns,
                           uint32_t* skey, uint64_t* smask, uint32_t* rkey, uint64_t* rmask,
                           uint32_t* tkey, uint64_t* tmask, uint32_t* l_key, uint64_t* l_mask,
                           uint32_t lds_cap, uint32_t* sel_hist = nullptr,
                           uint32_t* sel_state = nullptr) {
  const uint32_t rn = P->rec_count;
  __syncthreads();
  if (ns > 0) {
    const uint32_t nn = min((uint32_t)S, rn + ns);
    const uint32_t tot = rn + ns;
    if (tot <= kRankByCount && tot <= lds_cap) {
      // few entries: the record and the survivors side by side in LDS, each
      // entry's rank counted against all of them
      for (uint32_t t = threadIdx.x; t < tot; t += blockDim.x) {
        const bool in_rec = t < rn;
        l_key[t] = in_rec ? rkey[t] : skey[t - rn];
        l_mask[t] = in_rec ? rmask[t] : smask[t - rn];
      }
      __syncthreads();
      for (uint32_t t = threadIdx.x; t < tot; t += blockDim.x) {
        const uint32_t kx = l_key[t];
        const uint64_t mx = l_mask[t];
        uint32_t r = 0;
        for (uint32_t u = 0; u < tot; ++u) r += key_less(l_key[u], l_mask[u], kx, mx) ? 1u : 0u;
        if (r < nn) { tkey[r] = kx; tmask[r] = mx; }
      }
    } else {
      uint32_t nsort = ns;  // survivors that enter the sort
      bool gathered = false;
      if (sel_hist && ns > lds_cap && (uint32_t)S < lds_cap) {
        const uint32_t kS = radix_select(skey, ns, (uint32_t)S, sel_hist, sel_state);
        if (threadIdx.x == 0) sel_state[2] = 0u;
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < ns; c += blockDim.x) {
          const uint32_t key = skey[c];
          if (key <= kS) {
            const uint32_t slot = atomicAdd(&sel_state[2], 1u);
            if (slot < lds_cap) {
              l_key[slot] = key;
              l_mask[slot] = smask[c];
            }
          }
        }
        __syncthreads();
        const uint32_t ng = sel_state[2];
        if (ng <= lds_cap) {
          gathered = true;
          nsort = ng;
        }
        __syncthreads();
      }
      uint32_t P2 = 1;
      while (P2 < nsort) P2 <<= 1;
      uint32_t* ks;
      uint64_t* ms;
      if (gathered) {
        for (uint32_t t = nsort + threadIdx.x; t < P2; t += blockDim.x) {
          l_key[t] = 0xFFFFFFFFu;
          l_mask[t] = ~0ull;
        }
        ks = l_key;
        ms = l_mask;
      } else if (P2 <= lds_cap) {
        for (uint32_t t = threadIdx.x; t < P2; t += blockDim.x) {
          l_key[t] = t < ns ? skey[t] : 0xFFFFFFFFu;
          l_mask[t] = t < ns ? smask[t] : ~0ull;
        }
        ks = l_key;
        ms = l_mask;
      } else {
        for (uint32_t t = ns + threadIdx.x; t < P2 && t < cap; t += blockDim.x) {
          skey[t] = 0xFFFFFFFFu;
          smask[t] = ~0ull;
        }
        ks = skey;
        ms = smask;
      }
      __syncthreads();
      bitonic_sort(ks, ms, P2);
      for (uint32_t a = threadIdx.x; a < rn; a += blockDim.x) {
        const uint32_t r = a + rank_in(ks, ms, nsort, rkey[a], rmask[a]);
        if (r < nn) { tkey[r] = rkey[a]; tmask[r] = rmask[a]; }
      }
      for (uint32_t c = threadIdx.x; c < nsort; c += blockDim.x) {
        const uint32_t r = c + rank_in(rkey, rmask, rn, ks[c], ms[c]);
        if (r < nn) { tkey[r] = ks[c]; tmask[r] = ms[c]; }
      }
    }
    __syncthreads();
    for (uint32_t a = threadIdx.x; a < nn; a += blockDim.x) {
      rkey[a] = tkey[a];
      rmask[a] = tmask[a];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      P->rec_count = nn;
      if (nn == (uint32_t)S) {
        P->thr_key = rkey[S - 1];
        P->thr_mask = rmask[S - 1];
      }
    }
  }
  if (threadIdx.x == 0) {
    const uint32_t cc = P->cand_count;
    // overflow: the first cap candidates were merged, which can only lower
    // the threshold; the chunk is walked again unless this was the last pass
    P->redo = cc > cap ? 1u : 0u;
    if (cc > cap && !last_pass) P->stat_redo += 1;
    if (cc > cap && last_pass) P->err |= kErrCapacity;
    P->stat_candidates += cc;
    P->max_chunk_cand = max(P->max_chunk_cand, cc);
    P->cand_count = 0;
    P->surv_count = 0;
  }
}

// Single instance: one workgroup merges the survivors k_score left.
__global__ __launch_bounds__(kMergeThreads) void k_merge(Batch bt, int b, int retry,
                                                        int last_pass) {
  __shared__ uint32_t l_key[kLdsSortCap];
  __shared__ uint64_t l_mask[kLdsSortCap];
  __shared__ uint32_t sel_hist[256];
  __shared__ uint32_t sel_state[3];
  Params* P = bt.P + b;
  if (retry && !P->redo) return;
  const uint32_t ns = P->surv_count;
  merge_body(P, bt.S, bt.cap, last_pass != 0, ns, bt.skey + (size_t)b * bt.cap,
             bt.smask + (size_t)b * bt.cap, bt.rkey + (size_t)b * bt.S,
             bt.rmask + (size_t)b * bt.S, bt.tkey + (size_t)b * bt.S,
             bt.tmask + (size_t)b * bt.S, l_key, l_mask, (uint32_t)kLdsSortCap, sel_hist,
             sel_state);
}

// Batch: one workgroup per instance scores its own candidates of the chunk
// starting at first_mask, then merges the survivors into its record.  When
// there are many candidates, only those whose walk energy is within twice the
// margin of the S-th smallest walk energy are rescored: the walk energy is
// within the margin of the exact one, so the S-th smallest exact energy of the
// chunk is at most that S-th walk energy plus the margin, and no state at or
// below it can have a walk energy beyond twice the margin.  A chunk that
// overflowed its candidate buffer (and will be walked again) merges only
// the candidates of its S smallest walk energies.
template <bool kInt>
__global__ __launch_bounds__(kMergeBatchThreads) void k_merge_batched(Batch bt,
                                                                      uint64_t first_mask,
                                                                      int retry, int last_pass) {
  __shared__ uint32_t l_key[kLdsSortCapBatch];
  __shared__ uint64_t l_mask[kLdsSortCapBatch];
  __shared__ uint32_t s_inst[kMaxNBatched * kMaxNBatched + kMaxNBatched];
  __shared__ uint32_t s_hist[kMergeBatchThreads];
  __shared__ uint32_t s_sel[2];
  __shared__ uint32_t s_ns;
  __shared__ uint32_t s_list;
  const int b = blockIdx.x;
  const int N = inst_N(bt, b);
  if (N < kU || N > bt.ld || (N < 63 && first_mask >= (1ull << N))) return;
  Params* P = bt.P + b;
  if (retry && !P->redo) return;
  stage_instance<kInt>(bt, b, N, s_inst);
  if (threadIdx.x == 0) {
    s_ns = 0;
    s_list = 0;
  }
  __syncthreads();
  const uint64_t* cand = bt.cand + (size_t)b * bt.cap;
  const uint32_t* ckey = bt.ckey + (size_t)b * bt.cap;
  uint32_t* skey = bt.skey + (size_t)b * bt.cap;
  uint64_t* smask = bt.smask + (size_t)b * bt.cap;
  const uint32_t cnt = min(P->cand_count, bt.cap);
  const uint32_t thr_key = P->thr_key;
  const uint64_t thr_mask = P->thr_mask;
  const bool full = P->rec_count != 0 && thr_key != 0xFFFFFFFFu;
  uint32_t sel = 0xFFFFFFFFu;  // rescore candidates whose walk key is <= sel
  if (cnt > 2u * (uint32_t)bt.S + 256u) {
    const uint32_t kf = radix_select(ckey, cnt, (uint32_t)bt.S, s_hist, s_sel);
    // walk energies are exact, or the chunk overflowed and is walked again:
    // its S best walk energies lower the threshold for that pass, and what
    // they leave out is found then
    const bool again = P->cand_count > bt.cap && !last_pass;
    if (kInt || P->margin == 0.0f || again) {
      sel = kf;
    } else {
      const float ef = __uint_as_float(bits_of_f32_key(kf));
      sel = key_f32(f32_up((double)ef + 2.0 * (double)P->margin));
    }
  }
  // The preselected candidates are gathered in LDS (l_mask, free until the
  // merge) before they are rescored, so that the lanes of a wave rescore
  // one each: a rescoring costs O(N^2) and a wave pays it for any active
  // lane.  Windows of 2 x 256 candidates are scanned; the gathered ones are
  // rescored once there are 256 or at the end (at most 255 + 512 held).
  constexpr uint32_t kWin = 2 * kMergeBatchThreads;
  constexpr uint32_t kFlush = kMergeBatchThreads;
  static_assert(kFlush - 1 + kWin <= (uint32_t)kLdsSortCapBatch, "gather list exceeds l_mask");
  const uint32_t rn0 = P->rec_count;
  for (uint32_t w0 = 0; w0 < cnt; w0 += kWin) {
    const uint32_t w1 = min(cnt, w0 + kWin);
    for (uint32_t j = w0 + threadIdx.x; j < w1; j += blockDim.x) {
      const bool take = ckey[j] <= sel;
      const uint64_t act = __ballot(take);
      if (take) {  // one LDS atomic per wave
        const int lid = __lane_id();
        const int leader = __ffsll((unsigned long long)act) - 1;
        uint32_t base = 0;
        if (lid == leader) base = atomicAdd(&s_list, (uint32_t)__popcll(act));
        base = __shfl(base, leader);
        l_mask[base + (uint32_t)__popcll(act & ((1ull << lid) - 1ull))] = cand[j];
      }
    }
    __syncthreads();
    const uint32_t L = s_list;
    const bool flush = L >= kFlush || w1 == cnt;
    __syncthreads();  // every thread has read s_list
    if (flush) {
      if (threadIdx.x == 0) s_list = 0;
      for (uint32_t q = threadIdx.x; q < L; q += blockDim.x) {
        const uint64_t m = l_mask[q];
        const uint32_t key = exact_key<kInt>(s_inst, s_inst + N * N, N, N, m);
        bool keep = !full || key_less(key, m, thr_key, thr_mask);
        if (keep && retry)
          keep = !in_record(bt.rkey + (size_t)b * bt.S, bt.rmask + (size_t)b * bt.S, rn0, key, m);
        if (keep) {
          const uint32_t slot = atomicAdd(&s_ns, 1u);
          skey[slot] = key;
          smask[slot] = m;
        }
      }
      __syncthreads();  // l_mask read before the next window writes it
    }
  }
  const uint32_t ns = s_ns;
  merge_body(P, bt.S, bt.cap, last_pass != 0, ns, skey, smask, bt.rkey + (size_t)b * bt.S,
             bt.rmask + (size_t)b * bt.S, bt.tkey + (size_t)b * bt.S,
             bt.tmask + (size_t)b * bt.S, l_key, l_mask, (uint32_t)kLdsSortCapBatch);
}

// -------------------------------------------------------------- k_finalize
// grid.y indexes the instance; outputs are [B][S].

template <bool kInt>
__global__ void k_finalize(Batch bt, uint64_t* states_out, void* energies_out) {
  const int b = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const Params* P = bt.P + b;
  if (k == 0) atomicOr(bt.sticky, P->err);
  if (k >= bt.S) return;
  const size_t o = (size_t)b * bt.S + k;
  const bool have = (uint32_t)k < P->rec_count;
  const uint32_t key = have ? bt.rkey[(size_t)b * bt.S + k] : 0u;
  states_out[o] = have ? bt.rmask[(size_t)b * bt.S + k] : ~0ull;
  if (kInt) ((int32_t*)energies_out)[o] = have ? i32_of_key(key) : 0;
  else ((float*)energies_out)[o] = have ? __uint_as_float(bits_of_f32_key(key)) : 0.0f;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_prep(bool isint, const Batch& bt, hipStream_t st) {
  if (isint) hipLaunchKernelGGL(k_prep<true>, dim3(bt.B), dim3(256), 0, st, bt);
  else hipLaunchKernelGGL(k_prep<false>, dim3(bt.B), dim3(256), 0, st, bt);
  return hipGetLastError();
}

// records of n = U .. ncap (at table_base8 for U = kUWide)
// paired: also write the packed steps of the paired walk
hipError_t launch_tables(bool isint, int U, const Batch& bt, int ncap, bool paired,
                         hipStream_t st) {
  if ((U != kU && U != kUWide && U != kUPk) || ncap < U) return hipErrorInvalidValue;
  const int64_t total = ((int64_t)1 << (ncap - U + 1)) - 1;  // search records
  const dim3 grid((unsigned)((total + 255) / 256), (unsigned)bt.B);
#define SG_TABLES(I, UV) \
  hipLaunchKernelGGL((k_tables<I, false, UV>), grid, dim3(256), 0, st, bt, ncap, nullptr, \
                     paired ? 1 : 0)
  if (isint) {
    if (U == kU) SG_TABLES(true, kU);
    else if (U == kUWide) SG_TABLES(true, kUWide);
    else SG_TABLES(true, kUPk);
  } else {
    if (U == kU) SG_TABLES(false, kU);
    else if (U == kUWide) SG_TABLES(false, kUWide);
    else SG_TABLES(false, kUPk);
  }
#undef SG_TABLES
  return hipGetLastError();
}

// fp64 records (2 + U doubles each) of an fp32 batch, for the log Z walk.
hipError_t launch_tables64(const Batch& bt, int ncap, int U, double* out, hipStream_t st) {
  if (U != kLzU && U != kLzUF && U != kLzUW) return hipErrorInvalidValue;
  const int64_t total = ((int64_t)1 << (ncap - U + 1)) - 1;
  const dim3 grid((unsigned)((total + 255) / 256), (unsigned)bt.B);
  if (U == kLzUW)
    hipLaunchKernelGGL((k_tables<false, true, kLzUW>), grid, dim3(256), 0, st, bt, ncap, (void*)out,
                       0);
  else if (U == kLzU)
    hipLaunchKernelGGL((k_tables<false, true, kLzU>), grid, dim3(256), 0, st, bt, ncap, (void*)out,
                       0);
  else
    hipLaunchKernelGGL((k_tables<false, true, kLzUF>), grid, dim3(256), 0, st, bt, ncap, (void*)out,
                       0);
  return hipGetLastError();
}

// The paired walk takes the chunks (single searches) and levels (batches)
// with blocks of kUWide and at least two high spins (its tables hold the
// packed steps of those n); blocks of kUPk always walk paired (n >= kUPk + 2).
bool enum_paired(int U, int n) {
  return (U == kUWide && n >= kUWide + 2) || (U == kUPk && n >= kUPk + 2);
}

// The chunks the host marks (blocks of kUPk, n >= kUPk + kTriMinM, a single
// search's tables with packed triples) take the three-field walk.
bool enum_tri(bool split, const Batch& bt, const Chunk& ch) {
  return !split && bt.tri && ch.tri && ch.n >= kUPk + kTriMinM;
}

// split: test the bound per 64-step sub-block (batched searches)
hipError_t launch_enum(bool isint, int U, bool split, const Batch& bt, const Chunk& ch, int ninst,
                       hipStream_t st) {
  if ((U != kU && U != kUWide && U != kUPk) || ch.n < U) return hipErrorInvalidValue;
  if (U == kUPk && !enum_paired(U, ch.n)) return hipErrorInvalidValue;
  const int bpi = (int)((ch.lanes + kEnumBlock - 1) / kEnumBlock);
  const dim3 grid((unsigned)((int64_t)bpi * ninst));
#define SG_ENUM_T(I, UV, SP, PK, TR)                                                           \
  hipLaunchKernelGGL((k_enum<I, UV, SP, PK, TR>), grid, dim3(kEnumBlock), 0, st, bt, bt.J, bt.h, \
                     (const uint32_t*)bt.table, (const uint32_t*)bt.qtab, ch, bpi)
#define SG_ENUM(I, UV, SP, PK) SG_ENUM_T(I, UV, SP, PK, false)
#define SG_ENUM_U(I, SP)                 \
  if (U == kU) SG_ENUM(I, kU, SP, false); \
  else SG_ENUM(I, kUWide, SP, false)
  if (U == kUPk && enum_tri(split, bt, ch)) {
    if (isint) SG_ENUM_T(true, kUPk, false, true, true);
    else SG_ENUM_T(false, kUPk, false, true, true);
  } else if (U == kUPk) {
    if (isint) {
      if (split) SG_ENUM(true, kUPk, true, true);
      else SG_ENUM(true, kUPk, false, true);
    } else {
      if (split) SG_ENUM(false, kUPk, true, true);
      else SG_ENUM(false, kUPk, false, true);
    }
  } else if (enum_paired(U, ch.n)) {
    if (isint) {
      if (split) SG_ENUM(true, kUWide, true, true);
      else SG_ENUM(true, kUWide, false, true);
    } else {
      if (split) SG_ENUM(false, kUWide, true, true);
      else SG_ENUM(false, kUWide, false, true);
    }
  } else if (isint) {
    if (split) SG_ENUM_U(true, true);
    else SG_ENUM_U(true, false);
  } else {
    if (split) SG_ENUM_U(false, true);
    else SG_ENUM_U(false, false);
  }
#undef SG_ENUM_U
#undef SG_ENUM
#undef SG_ENUM_T
  return hipGetLastError();
}

hipError_t launch_direct(const Batch& bt, uint64_t lo, uint64_t hi, hipStream_t st) {
  const uint64_t cnt = hi - lo;
  hipLaunchKernelGGL(k_direct, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, bt, lo, hi);
  return hipGetLastError();
}

hipError_t launch_score(bool isint, const Batch& bt, int b, int grid, int N, int retry,
                        hipStream_t st) {
  const size_t shm = (size_t)(N * N + N) * 4;
  if (isint) hipLaunchKernelGGL(k_score<true>, dim3(grid), dim3(256), shm, st, bt, b, retry);
  else hipLaunchKernelGGL(k_score<false>, dim3(grid), dim3(256), shm, st, bt, b, retry);
  return hipGetLastError();
}

hipError_t launch_merge(const Batch& bt, int b, int retry, bool last_pass, hipStream_t st) {
  hipLaunchKernelGGL(k_merge, dim3(1), dim3(kMergeThreads), 0, st, bt, b, retry,
                     last_pass ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_merge_batched(bool isint, const Batch& bt, uint64_t first_mask, int retry,
                                bool last_pass, hipStream_t st) {
  if (isint)
    hipLaunchKernelGGL(k_merge_batched<true>, dim3(bt.B), dim3(kMergeBatchThreads), 0, st, bt,
                       first_mask, retry, last_pass ? 1 : 0);
  else
    hipLaunchKernelGGL(k_merge_batched<false>, dim3(bt.B), dim3(kMergeBatchThreads), 0, st, bt,
                       first_mask, retry, last_pass ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_finalize(bool isint, const Batch& bt, uint64_t* states_out, void* energies_out,
                           hipStream_t st) {
  const dim3 grid((unsigned)((bt.S + 255) / 256), (unsigned)bt.B);
  if (isint)
    hipLaunchKernelGGL(k_finalize<true>, grid, dim3(256), 0, st, bt, states_out, energies_out);
  else
    hipLaunchKernelGGL(k_finalize<false>, grid, dim3(256), 0, st, bt, states_out, energies_out);
  return hipGetLastError();
}

// resident workgroups per CU of the walk (the smallest over its variants)
template <bool I>
int enum_occupancy_t() {
  int best = 1 << 30;
  auto take = [&](const void* f) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, kEnumBlock, 0) != hipSuccess)
      blocks = 0;
    best = blocks < best ? blocks : best;
  };
  take((const void*)k_enum<I, kU, false, false>);
  take((const void*)k_enum<I, kUWide, false, false>);
  take((const void*)k_enum<I, kU, true, false>);
  take((const void*)k_enum<I, kUWide, true, false>);
  take((const void*)k_enum<I, kUWide, false, true>);
  take((const void*)k_enum<I, kUWide, true, true>);
  take((const void*)k_enum<I, kUPk, false, true, true>);
  take((const void*)k_enum<I, kUPk, false, true>);
  take((const void*)k_enum<I, kUPk, true, true>);
  return best;
}

int enum_occupancy(bool isint) {
  return isint ? enum_occupancy_t<true>() : enum_occupancy_t<false>();
}

}  // namespace sg
