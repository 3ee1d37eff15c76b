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

// Low spins per search block: U = kUWide (2^8 = 256 steps) wherever a lane
// has at least 8 free spins (single searches of N >= 16, batch levels of
// n >= 8), which spreads the per-block set-up over twice the states of
// U = kU (2^7 = 128 steps), the size taken otherwise and by the density of
// states.
constexpr int kU = 7;
constexpr int kUWide = 8;
// The paired walk of a single search takes blocks of kUPk = 10 (2^10 steps)
// where a lane has at least kUPk + 2 free spins and the walk is in fp32: its
// per-block work (fixed-point start values, fp32 G updates, record reads,
// the bound test) then comes once per 2^10 steps instead of 2^8.
constexpr int kUPk = 10;
constexpr int kBlockSteps = 1 << kU;
// qtab words per instance: the tables of U = kU (both block parities), then
// those of U = kUWide, then those of U = kUPk (single searches only)
constexpr int kQStride = (2 << kU) + (2 << kUWide) + (2 << kUPk);
constexpr int qtab_base(int U) {
  return U == kUPk ? (2 << kU) + (2 << kUWide) : U == kUWide ? (2 << kU) : 0;
}
// index of a block size's Q minimum in Params::qmin_f / qmin_i
constexpr int qmin_index(int U) { return U == kUPk ? 2 : U == kUWide ? 1 : 0; }
constexpr int kMaxFree = 22;          // largest n (free spins per lane)
constexpr int kMaxHigh = kMaxFree - kU;
constexpr int kRecWords = 16;         // per-block table record (64 B: cB, R, Wu_0..U-1, U <= 14)
// records of the blocks of kUPk: 32 words (128 B), every packed step in the
// first record of a pair
constexpr int rec_words(int U) { return U == kUPk ? 32 : kRecWords; }
constexpr int kReanchorLog2 = 10;     // fp32: fresh G every 2^10 flips
constexpr int kReanchorBlocks = 1 << (kReanchorLog2 - kU);
// The paired walk carries G in fp32 only from block to block (a boundary step
// of two rounded adds, the block's net step of two, and the two roundings of
// that step's value: 6 per block of 2^kUWide flips), so it re-anchors every
// 2^14 flips and stays inside the rounding count the margin allows between
// anchors for the plain walk (2^(10 - U) (2^U - 1 + 3U + 3) with U = kUWide).
constexpr int kPkReanchorLog2 = 14;
static_assert((1 << (kPkReanchorLog2 - kUWide)) * 6 <=
                  (1 << (kReanchorLog2 - kUWide)) * ((1 << kUWide) - 1 + 3 * kUWide + 3),
              "paired-walk re-anchor period exceeds the margin's rounding count");
static_assert((1 << (kPkReanchorLog2 - kUPk)) * 6 <=
                  (1 << (kReanchorLog2 - kUWide)) * ((1 << kUWide) - 1 + 3 * kUWide + 3),
              "paired-walk re-anchor period exceeds the margin's rounding count");
// The log Z walk uses blocks of its own, U low spins with fp64 records of
// 2 + U doubles (cB, R, Wu_0..U-1): the partition sums take U = 10 (1024
// configurations) when N >= 10 and at most three beta, else U = 8 when
// N >= 8; the gradient walk U = 8 (four sub-blocks of 6) when N >= 8; N = 7
// takes U = 6 in both.
constexpr int kLzU = 6;
constexpr int kLzUF = 8;
constexpr int kLzUW = 10;  // the partition sums' records when N >= 10
constexpr int kLzSteps = 1 << kLzU;
// floats per (instance, beta) of the bq tables: 256 up to records of 8, 1024
// for records of 10 (the same buffer, [B][kMaxBeta][stride])
constexpr int lz_q_stride(int U) { return U > kLzUF ? 1 << U : 1 << kLzUF; }
constexpr int kLzQStride = lz_q_stride(kLzUW);  // the buffer's floats per (instance, beta)
// Bytes of the static device array that the allocation-free log Z backward
// takes its buffers from (one array per device, held until the process ends).
constexpr unsigned long long kLzScratchBytes = 32ull << 20;
constexpr int kWaveLanes = 64;
constexpr int kEnumBlock = 256;       // threads per enumeration workgroup
constexpr int kMergeThreads = 1024;   // threads of the single-workgroup merge
constexpr int kMergeBatchThreads = 256;  // threads per instance in the batched merge
constexpr int kBatchFreeCap = 16;     // largest n of a batched search
constexpr int kLdsSortCap = 4096;     // survivors sorted in LDS up to this
constexpr int kLdsSortCapBatch = 1024;  // the same for the per-instance batched merge
constexpr int kRankByCount = 512;     // merges of up to this many entries rank by counting
constexpr int kQuboSortCap = 4096;    // states of a QUBO search (sorted in LDS)
constexpr int kMaxN = 63;            // largest N (masks are 64-bit, signed in the bindings)
constexpr int kMaxNBatched = 40;     // largest N_max of a batched search

// Sticky device error bits (mapped to sg_status on the host).
enum : uint32_t {
  kErrNonFinite = 1u << 0,
  kErrOverflow = 1u << 1,
  kErrCapacity = 1u << 2,
  kErrDrift = 1u << 3,
  kErrInval = 1u << 4,   // device-side argument check (batched N_b, S)
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
  float qmin_f[3];       // min over low configs of Q (rounded down), [qmin_index(U)]
  int32_t qmin_i[3];
  uint32_t err;          // sticky error bits
  // per-chunk counters
  uint32_t cand_count;   // candidates appended by the current chunk
  uint32_t surv_count;   // candidates that beat the threshold after rescoring
  // statistics
  unsigned long long stat_candidates;
  unsigned long long stat_slow;
  uint32_t max_drift_bits;  // float bits, non-negative
  uint32_t max_chunk_cand;  // most candidates any one chunk produced
  // 1 when the last pass over the current chunk produced more candidates
  // than the buffer holds: the chunk is walked again with the tightened
  // threshold (at most kRetries times)
  uint32_t redo;
  uint32_t walk_f32;         // integer instance walked in fp32 (exact: |values| < 2^24)
  uint32_t stat_redo;       // repeated passes taken
  double bound;             // sum_{i<j} |J_ij| + sum_i |h_i| (no |E| exceeds it)
  // paired walk (two 16-bit fixed-point fields per word): the power-of-two
  // scale of its values (0: not available), and the slack subtracted from the
  // field offset 2^15 so that rounding never hides a state below the bound
  float pk_scale;
  int32_t pk_slack;
  float pk_scale10;      // the same for the blocks of kUPk (slack kUPk + 1)
  int32_t pk_slack10;
  // three-field walk (blocks of kUPk, single searches): the power-of-two
  // scale of its values, and the part of the bound on a block's summed step
  // magnitudes (units) that does not depend on the lane
  float pk_scale3;
  int32_t pk_rb3;
};

// Three-field walk: chunks of a single search with n >= kUPk + kTriMinM free
// spins may walk three blocks of kUPk at once, as the fields of one 32-bit
// word (bits 0-10, 11-21 and 22-31); the host picks it per chunk (Chunk::tri).
// A lane's 2^m blocks (m = n - kUPk) are taken
// in levels: level l holds the triples (b + T, b + Q + T, b + 2Q + T), T < Q,
// with Q = 2^(m - 2 - 2l) >= 2 and b = 2^m - 4Q; the 2 or 4 blocks left
// after the last level are walked exactly.  The record of b + T holds the
// triple's packed record steps, from word kPkWordTri (the paired walk's stay
// in words pk_word(kUPk) ..., so either walk can take the chunk).  Every field keeps a margin of kTriRoom
// units on both sides of its test bit (the 10-bit field sets the limit).
constexpr int kTriMinM = 4;
constexpr int kTriShiftB = 11;
constexpr int kTriShiftC = 22;
constexpr int kTriRoom = 512;  // half the range of the 10-bit field
constexpr uint32_t kTriBias = 1024u + (1024u << kTriShiftB) + (512u << kTriShiftC);
constexpr uint32_t kTriLane = 1u + (1u << kTriShiftB) + (1u << kTriShiftC);
// blocks of a lane with 2^m blocks that the levels cover (the rest, 2 or 4,
// is the exact tail)
__host__ __device__ constexpr uint32_t tri_covered(int m) {
  return (1u << m) - ((m & 1) ? 2u : 4u);
}

// Paired walk: the record of block T < half of a table (n >= U + 2 free
// spins, U = kUWide or kUPk) holds, from word pk_word(U), the packed record
// steps pk_f = (Wx_f(T + half) << 16) + Wx_f(T) (integer sum mod 2^32, Wx the
// fixed-point value of the record's Wu_f) of f < pk_in_a(U); with U = kUWide
// the record of block T + half holds f = 6, 7 in its words pk_word(U) + 0, 1.
constexpr int pk_word(int U) { return 2 + U; }
constexpr int pk_in_a(int U) { return U == kUPk ? U : kRecWords - pk_word(U); }
constexpr int kPkWordTri = pk_word(kUPk) + kUPk;  // the three-field walk's packed steps
static_assert(kPkWordTri + kUPk <= rec_words(kUPk), "triple steps exceed the record");
static_assert(pk_word(kUPk) + kUPk <= rec_words(kUPk), "packed steps exceed the record");
static_assert(pk_word(kUWide) + kUWide <= 2 * kRecWords - pk_word(kUWide), "packed steps split");

// Extra passes over a chunk whose candidates overflowed the buffer.
constexpr int kRetries = 2;

// Device views of one search over B instances (B = 1 for a single search).
// Instance b has N_b spins (Ns[b], or N0 for every instance when Ns is
// null); its couplings are J[b][i][j] with row stride ld (i < j read), its
// fields h[b][i].  Every per-instance buffer is a slice of a [B][...] array.
struct Batch {
  const void* J;
  const void* h;
  const int32_t* Ns;
  int N0;
  int ld;
  int B;
  int S;
  Params* P;           // [B]
  uint32_t* qtab;      // [B][kQStride] low-low energies by block parity and step
  uint32_t* table;     // [B][table_recs][kRecWords]
  int64_t table_recs;
  int64_t table_base10w;  // first word of the U = kUPk tables (single searches)
  int64_t table_base8; // first record of the U = kUWide tables (search tables)
  uint64_t* cand;      // [B][cap] candidate masks
  uint32_t* ckey;      // [B][cap] orderable key of each candidate's walk energy
  uint32_t* skey;      // [B][cap]
  uint64_t* smask;     // [B][cap]
  uint32_t cap;
  uint32_t* rkey;      // [B][S] record: keys ascending
  uint64_t* rmask;     // [B][S]
  uint32_t* tkey;      // [B][S] merge scratch
  uint64_t* tmask;     // [B][S]
  uint32_t* sticky;    // error bits accumulated over searches
  int allow_f32_walk;  // integer instances may take the fp32 walk (searches: 1)
  int tri;             // single searches: tables of n >= kUPk + kTriMinM hold triples
  float margin_scale;  // factor on the fp32 pruning margin (1; test hook only)
};

// Exact log Z walk (forward: partition sums; backward: gradient moments).
constexpr int kMaxBeta = 4;
constexpr int kLzFree = 14;  // free spins per lane: n = min(N, 14)

struct LzArgs {
  int B, N, n, nb, S;
  int U;                // low spins per block (kLzU or kLzUF)
  int64_t lanes;        // lanes per instance: 2^(N - n)
  int64_t table_recs;   // fp64 records per instance
  int table_offset;     // first record of the table of n
  const float* h_in;    // [B][N] fields
  const float* beta;    // [nb]
  const float* e0;      // [B] shift (ground energy)
  double* coef;         // [B][2][kMaxBeta]: backward weights g_b beta_b / Z_b, then
                        // -beta_b / ln 2
  double* acc;          // forward: [B][kMaxBeta]; backward: [B][N*N + N]
  int acc_stride;
  uint32_t* sticky;
};

// One enumeration launch: lanes L, prefixes base..base+L-1, n free spins.
struct Chunk {
  uint64_t first_mask;    // = base << n
  uint64_t prefix_base;
  int64_t lanes;
  int n;
  int table_offset;       // record index of block 0 in the table for this n
  int table_offset8;      // the same in the U = kUWide table, for a chunk of
                          // U = kUPk whose instance takes the int32 walk
  int retry;              // 0: first pass; r >= 1: r-th repeat (only if redo)
  int tri;                // blocks of kUPk: the three-field walk (n >= kUPk + kTriMinM)
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
