// sg_dos.hip -- exact density of states of an integer instance: the number of
// configurations at every energy of Eq. (1), all 2^N states enumerated.
//
// The walk is the search's decomposition (one lane per prefix, free spins in
// Gray-code order, blocks of 2^U steps with the low-low energies Q in a
// per-parity table) in int32, so every state's energy is exact.  A state costs
// one add for its energy and one LDS atomic increment of its bin; energies and
// fields are kept scaled by 4 so that the bin's byte offset is the sum itself.
// Each workgroup owns an LDS histogram (32-bit: a workgroup sees at most
// 256 * 2^22 states) and adds its non-zero bins to the 64-bit global counts.
// The lanes of a wave tend to fall into a few bins at once, and increments of
// one LDS word serialise; so the histogram is held in R copies interleaved
// word by word (bin k of copy c at word k R + c), lane l using copy l mod R:
// lanes that meet in one bin mostly hit different words and banks.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_internal.h"

namespace sg {

// counts[0 .. n_bins) = 0 (a fill kernel: the sequence records no memset)
__global__ void k_dos_zero(unsigned long long* counts, int n_bins) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_bins) counts[k] = 0ull;
}

// The instance's energy bound sum_{i<j} |J_ij| + sum_i |h_i| (int64), one
// workgroup.
__global__ void k_energy_bound(int N, const int32_t* __restrict__ J, const int32_t* __restrict__ h,
                               long long* out) {
  __shared__ long long s[256];
  long long acc = 0;
  for (int k = threadIdx.x; k < N * N + N; k += blockDim.x) {
    if (k < N * N) {
      if (k / N < k % N) acc += llabs((long long)J[k]);
    } else {
      acc += llabs((long long)h[k - N * N]);
    }
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// After k_prep: the bins must cover [-B, B] (B the energy bound, which no
// energy exceeds in size); the instance's error bits go to the sticky word.
__global__ void k_dos_check(Batch bt, long long e_min, int n_bins) {
  Params* P = bt.P;
  uint32_t err = P->err;
  const double B = P->bound;
  if ((double)e_min > -B || (double)e_min + (double)(n_bins - 1) < B) err |= kErrInval;
  P->err = err;
  if (err) atomicOr(bt.sticky, err);
}

__global__ __launch_bounds__(256) void k_dos(Batch bt, const int32_t* __restrict__ J,
                                             const int32_t* __restrict__ h,
                                             const uint32_t* __restrict__ table,
                                             const uint32_t* __restrict__ qtab, Chunk ch,
                                             long long e_min, int n_bins, int rep,
                                             unsigned long long* counts) {
  constexpr int U = kU;
  extern __shared__ uint32_t s_hist[];  // n_bins * rep counters
  __shared__ int32_t s_y[kMaxHigh * 256];
  const Params* P = bt.P;
  if (P->err) return;  // uniform: bad instance or bins

  const int N = bt.N0, n = ch.n, tid = threadIdx.x;
  for (int k = tid; k < n_bins * rep; k += 256) s_hist[k] = 0u;
  const int64_t lane = (int64_t)blockIdx.x * 256 + tid;
  const bool valid = lane < ch.lanes;
  const uint64_t p = ch.prefix_base + (uint64_t)(valid ? lane : 0);
  const uint32_t* tab = table + (size_t)ch.table_offset * kRecWords;

  // per-lane init, exact: y_f = sum_q J_fq s_q over the prefix spins q >= n;
  // WL_f = 2 y_f for the low spins, Y_g = 2 y_g (LDS) for the high ones; E_P
  int32_t WL[U];
  int32_t ysum = 0;
#pragma unroll
  for (int f = 0; f < U; ++f) {
    int32_t acc = 0;
    for (int q = n; q < N; ++q) {
      const int32_t jq = J[f * N + q];
      acc += ((p >> (q - n)) & 1ull) ? jq : -jq;
    }
    ysum += acc;
    WL[f] = 2 * acc;
  }
  for (int f = U; f < n; ++f) {
    int32_t acc = 0;
    for (int q = n; q < N; ++q) {
      const int32_t jq = J[f * N + q];
      acc += ((p >> (q - n)) & 1ull) ? jq : -jq;
    }
    ysum += acc;
    s_y[(f - U) * 256 + tid] = 2 * acc;
  }
  int32_t EP = 0;
  for (int q = n; q < N; ++q) {
    const int32_t sq = ((p >> (q - n)) & 1ull) ? 1 : -1;
    int32_t f = h[q];
    for (int r = q + 1; r < N; ++r) {
      const int32_t jr = J[q * N + r];
      f += ((p >> (r - n)) & 1ull) ? jr : -jr;
    }
    EP -= sq * f;
  }
  // Byte offset 4 (R (E - e_min) + c) of the state's counter without the
  // low-low part, at the first state; every energy term is scaled by 4R.  The
  // sums are taken modulo 2^32 (unsigned): intermediate values may leave the
  // int32 range, the offset of every state's counter does not.
  const uint32_t sc = 4u * (uint32_t)rep;  // byte stride of one bin
  uint32_t G4 = sc * ((uint32_t)EP + (uint32_t)ysum + tab[1] - (uint32_t)e_min) +
                4u * ((uint32_t)tid & (uint32_t)(rep - 1));
  __syncthreads();  // s_hist cleared, s_y written

  if (valid) {
    const uint32_t nblocks = 1u << (n - U);
    for (uint32_t T = 0; T < nblocks; ++T) {
      const uint32_t* rec = tab + (size_t)T * kRecWords;
      if (T != 0) {
        // boundary step: high spin U + c flips, old value +1 iff bit c+1 of T
        const int c = __builtin_ctz(T);
        const bool up = (T >> (c + 1)) & 1u;
        const uint32_t y4 = sc * (uint32_t)s_y[c * 256 + tid];
        G4 = up ? G4 + y4 : G4 - y4;
        G4 += sc * rec[0];
      }
      uint32_t W4[U];
#pragma unroll
      for (int f = 0; f < U - 1; ++f) W4[f] = sc * ((uint32_t)WL[f] + rec[2 + f]);
      W4[U - 1] = sc * ((uint32_t)((T & 1u) ? WL[U - 1] : -WL[U - 1]) + rec[2 + U - 1]);
      const uint32_t* q = qtab + (T & 1u) * kBlockSteps;
      atomicAdd((uint32_t*)((char*)s_hist + (G4 + sc * q[0])), 1u);
#pragma unroll
      for (int i = 1; i < kBlockSteps; ++i) {
        const int f = __builtin_ctz(i);
        if (f == U - 1) G4 += W4[f];
        else G4 = ((i >> (f + 1)) & 1) ? G4 + W4[f] : G4 - W4[f];
        atomicAdd((uint32_t*)((char*)s_hist + (G4 + sc * q[i])), 1u);
      }
    }
  }
  __syncthreads();
  for (int k = tid; k < n_bins; k += 256) {
    uint32_t c = 0u;
    for (int r = 0; r < rep; ++r) c += s_hist[k * rep + r];
    if (c) atomicAdd(counts + k, (unsigned long long)c);
  }
}

// Tiny instances (N < U): one thread per state, energy from scratch.
__global__ void k_dos_direct(Batch bt, const int32_t* __restrict__ J,
                             const int32_t* __restrict__ h, long long e_min,
                             unsigned long long* counts) {
  if (bt.P->err) return;
  const int N = bt.N0;
  const uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= (1ull << N)) return;
  int32_t e = 0;
  for (int i = 0; i < N; ++i) {
    const int32_t si = ((m >> i) & 1ull) ? 1 : -1;
    int32_t f = h[i];
    for (int j = i + 1; j < N; ++j) f += ((m >> j) & 1ull) ? J[i * N + j] : -J[i * N + j];
    e -= si * f;
  }
  atomicAdd(counts + (e - e_min), 1ull);
}

// ---------------------------------------------------------------- launchers

hipError_t launch_dos_prologue(const Batch& bt, long long e_min, int n_bins,
                               unsigned long long* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_dos_zero, dim3((n_bins + 255) / 256), dim3(256), 0, st, counts, n_bins);
  hipLaunchKernelGGL(k_dos_check, dim3(1), dim3(1), 0, st, bt, e_min, n_bins);
  return hipGetLastError();
}

// Copies of the histogram: the largest power of two up to 32 that keeps it
// within 32 KB of LDS.
int dos_copies(int n_bins) {
  int rep = 32;
  while (rep > 1 && (size_t)n_bins * rep * sizeof(uint32_t) > (32u << 10)) rep >>= 1;
  return rep;
}

hipError_t launch_dos(const Batch& bt, const Chunk& ch, long long e_min, int n_bins,
                      unsigned long long* counts, hipStream_t st) {
  const dim3 grid((unsigned)((ch.lanes + 255) / 256));
  const int rep = dos_copies(n_bins);
  const size_t shm = (size_t)n_bins * rep * sizeof(uint32_t);
  hipLaunchKernelGGL(k_dos, grid, dim3(256), shm, st, bt, (const int32_t*)bt.J,
                     (const int32_t*)bt.h, (const uint32_t*)bt.table, (const uint32_t*)bt.qtab, ch,
                     e_min, n_bins, rep, counts);
  return hipGetLastError();
}

hipError_t launch_dos_direct(const Batch& bt, long long e_min, unsigned long long* counts,
                             hipStream_t st) {
  const uint64_t states = 1ull << bt.N0;
  hipLaunchKernelGGL(k_dos_direct, dim3((unsigned)((states + 255) / 256)), dim3(256), 0, st, bt,
                     (const int32_t*)bt.J, (const int32_t*)bt.h, e_min, counts);
  return hipGetLastError();
}

hipError_t launch_energy_bound(int N, const int32_t* J, const int32_t* h, long long* out,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_energy_bound, dim3(1), dim3(256), 0, st, N, J, h, out);
  return hipGetLastError();
}

}  // namespace sg
