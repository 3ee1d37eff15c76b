// sg_internal.h -- definitions shared by the HIP kernels and the host side of
// the library (not part of the public ABI).
//
// Decomposition used by the enumeration (all symbols per instance):
//   spins 0..n-1 are "free" and walked by a reflected Gray code that is the
//   same for every lane; spins n..N-1 are the lane's fixed prefix p (the
//   thread-index encoding of Eqs. (4)-(6) applied to the top k = N - n bits).
//   The free spins split into the U lowest ("low", flipped inside a block of
//   2^U steps) and the rest ("high", flipped once per block boundary).
//   For a state (p, T, i) -- prefix p, block T, step i inside the block --
//       E(p,T,i) = G(p,T,i) + Q(low config)
//   where Q is the energy of the couplings among the low spins only (a
//   2^U-entry table shared by all lanes) and G changes by +-W_f (f low) per
//   inner step and by +-Y_g + c(T) (g high) per block boundary.
#pragma once

#include <stdint.h>

namespace sg {

constexpr int kU = 6;                 // low spins per block: 2^6 = 64 steps
constexpr int kBlockSteps = 1 << kU;
constexpr int kMaxFree = 22;          // largest n (free spins per lane)
constexpr int kMaxHigh = kMaxFree - kU;
constexpr int kRecWords = 8;          // per-block table record (32 B)
constexpr int kReanchorLog2 = 16;     // fp32: fresh G every 2^16 flips
constexpr int kReanchorBlocks = 1 << (kReanchorLog2 - kU);
constexpr int kWaveLanes = 64;
constexpr int kEnumBlock = 256;       // threads per enumeration workgroup
constexpr int kMergeThreads = 1024;   // threads of the single-workgroup merge
constexpr int kLdsSortCap = 4096;     // survivors sorted in LDS up to this
constexpr int kMaxN = 56;

// Sticky device error bits (mapped to sg_status on the host).
enum : uint32_t {
  kErrNonFinite = 1u << 0,
  kErrOverflow = 1u << 1,
  kErrCapacity = 1u << 2,
  kErrDrift = 1u << 3,
};

// Per-search device state, written by the prep / merge kernels and read by
// the enumeration kernel.  Lives in the workspace.
struct Params {
  // threshold = key of the S-th record entry (0xFFFFFFFF: record not full)
  uint32_t thr_key;
  uint32_t rec_count;
  uint64_t thr_mask;
  // instance-derived
  float margin;          // fp32 pruning margin (bound on incremental error)
  float qmin_f;          // min over low configs of Q (rounded down)
  int32_t qmin_i;
  uint32_t err;          // sticky error bits
  // per-chunk counters
  uint32_t cand_count;   // candidates appended by the current chunk
  uint32_t surv_count;   // candidates that beat the threshold after rescoring
  // statistics
  unsigned long long stat_candidates;
  unsigned long long stat_slow;
  uint32_t max_drift_bits;  // float bits, non-negative
  uint32_t pad0;
};

// One enumeration launch: lanes L, prefixes base..base+L-1, n free spins.
struct Chunk {
  uint64_t first_mask;    // = base << n
  uint64_t prefix_base;
  int64_t lanes;
  int n;
  int table_offset;       // record index of block 0 in the table for this n
};

// Orderable 32-bit keys of energies.
__host__ __device__ inline uint32_t key_of_f32_bits(uint32_t b) {
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ inline uint32_t bits_of_f32_key(uint32_t k) {
  return (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
}
__host__ __device__ inline uint32_t key_of_i32(int32_t e) {
  return static_cast<uint32_t>(e) ^ 0x80000000u;
}
__host__ __device__ inline int32_t i32_of_key(uint32_t k) {
  return static_cast<int32_t>(k ^ 0x80000000u);
}

}  // namespace sg
