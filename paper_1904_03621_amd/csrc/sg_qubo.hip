// sg_qubo.hip -- QUBO front end (Sec. 2, Eqs. 2-3): the low spectrum of
//   F(q) = - sum_{i<j} a_ij q_i q_j - sum_i b_i q_i,   q_i in {0, 1},
// found by the Ising search on the instance Eq. (3) relates it to:
//   J_ij = a_ij / 4,   h_i = b_i / 2 + sum_{j != i} a_ij / 4,
// for which H(s) = F(q) + sum_i h_i - sum_{i<j} J_ij with q = (s + 1) / 2, i.e.
// bit i of a mask is q_i in both.  The S states found are rescored in the
// QUBO form (fp64, rounded once) and sorted by (F, mask).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_internal.h"

namespace sg {

// One workgroup: the Ising couplings and fields of the QUBO (a, b).
__global__ void k_qubo_to_ising(int N, const float* __restrict__ A, const float* __restrict__ b,
                                float* J, float* h) {
  for (int k = threadIdx.x; k < N * N; k += blockDim.x) {
    const int i = k / N, j = k % N;
    J[k] = i < j ? 0.25f * A[k] : 0.0f;  // a / 4 is exact in fp32
  }
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double s = 0.5 * (double)b[i];
    for (int j = 0; j < N; ++j) {
      if (j == i) continue;
      s += 0.25 * (double)(i < j ? A[i * N + j] : A[j * N + i]);
    }
    h[i] = (float)s;
  }
}

__device__ inline uint32_t qkey(float e) {
  if (e == 0.0f) e = 0.0f;  // -0 -> +0
  const uint32_t bits = __float_as_uint(e);
  return (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
}

// One workgroup of 1024 threads: F of each found state, then a bitonic sort
// of (key, mask) in LDS and the outputs.
__global__ __launch_bounds__(1024) void k_qubo_finish(int N, const float* __restrict__ A,
                                                      const float* __restrict__ b, int S,
                                                      const uint64_t* found, uint64_t* states_out,
                                                      float* energies_out) {
  __shared__ uint32_t s_key[kQuboSortCap];
  __shared__ uint64_t s_mask[kQuboSortCap];
  uint32_t P2 = 1;
  while (P2 < (uint32_t)S) P2 <<= 1;
  for (uint32_t t = threadIdx.x; t < P2; t += blockDim.x) {
    if (t < (uint32_t)S) {
      const uint64_t m = found[t];
      double f = 0.0;
      for (int i = 0; i < N; ++i) {
        if (!((m >> i) & 1ull)) continue;
        double fi = (double)b[i];
        for (int j = i + 1; j < N; ++j)
          if ((m >> j) & 1ull) fi += (double)A[i * N + j];
        f -= fi;
      }
      s_key[t] = qkey((float)f);
      s_mask[t] = m;
    } else {
      s_key[t] = 0xFFFFFFFFu;
      s_mask[t] = ~0ull;
    }
  }
  __syncthreads();
  for (uint32_t size = 2; size <= P2; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = threadIdx.x; t < P2 / 2; t += blockDim.x) {
        const uint32_t x = 2 * t - (t & (stride - 1)), y = x + stride;
        const bool asc = (x & size) == 0;
        const uint32_t kx = s_key[x], ky = s_key[y];
        const uint64_t mx = s_mask[x], my = s_mask[y];
        const bool gt = ky < kx || (ky == kx && my < mx);
        if (gt == asc) {
          s_key[x] = ky; s_key[y] = kx;
          s_mask[x] = my; s_mask[y] = mx;
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t t = threadIdx.x; t < (uint32_t)S; t += blockDim.x) {
    const uint32_t k = s_key[t];
    const uint32_t bits = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    states_out[t] = s_mask[t];
    energies_out[t] = __uint_as_float(bits);
  }
}

hipError_t launch_qubo_to_ising(int N, const float* A, const float* b, float* J, float* h,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_qubo_to_ising, dim3(1), dim3(256), 0, st, N, A, b, J, h);
  return hipGetLastError();
}

hipError_t launch_qubo_finish(int N, const float* A, const float* b, int S, const uint64_t* found,
                              uint64_t* states_out, float* energies_out, hipStream_t st) {
  hipLaunchKernelGGL(k_qubo_finish, dim3(1), dim3(1024), 0, st, N, A, b, S, found, states_out,
                     energies_out);
  return hipGetLastError();
}

}  // namespace sg
