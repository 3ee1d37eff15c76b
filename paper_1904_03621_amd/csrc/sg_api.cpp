// sg_api.cpp -- host side of the C ABI (include/sg.h): argument validation,
// per-(device, stream) workspace, the chunk plan and the kernel sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/sg.h"
#include "sg_internal.h"

namespace sg {
hipError_t launch_prep(bool isint, const Batch& bt, hipStream_t st);
hipError_t launch_tables(bool isint, int U, const Batch& bt, int ncap, bool paired,
                         hipStream_t st);
hipError_t launch_enum(bool isint, int U, bool split, const Batch& bt, const Chunk& ch, int ninst,
                       hipStream_t st);
hipError_t launch_direct(const Batch& bt, uint64_t lo, uint64_t hi, hipStream_t st);
hipError_t launch_score(bool isint, const Batch& bt, int b, int grid, int N, int retry,
                        hipStream_t st);
hipError_t launch_merge(const Batch& bt, int b, int retry, bool last_pass, hipStream_t st);
hipError_t launch_merge_batched(bool isint, const Batch& bt, uint64_t first_mask, int retry,
                                bool last_pass, hipStream_t st);
hipError_t launch_finalize(bool isint, const Batch& bt, uint64_t* states_out, void* energies_out,
                           hipStream_t st);
int enum_occupancy(bool isint);
double probe_valu(int op, int waves_per_simd);
hipError_t launch_tables64(const Batch& bt, int ncap, int U, double* out, hipStream_t st);
hipError_t launch_lz_prep(int mode, const LzArgs& a, const float* J, float* lzq, double* lzqmin,
                          const float* energies, float* e0_out, const double* logz,
                          const double* grad, hipStream_t st);
hipError_t launch_logz(int mode, const LzArgs& a, const float* J, const float* h,
                       const double* table64, const float* lzq, const double* lzqmin,
                       hipStream_t st);
hipError_t launch_lz_final(int mode, const LzArgs& a, double* logz, float* grad_J, float* grad_h,
                           hipStream_t st);
hipError_t lz_scratch(void** ptr, bool* fresh);
void* lz_scratch_resolved();
hipError_t launch_clear_word(uint32_t* p, hipStream_t st);
hipError_t launch_dos_prologue(const Batch& bt, long long e_min, int n_bins,
                               unsigned long long* counts, hipStream_t st);
hipError_t launch_dos(const Batch& bt, const Chunk& ch, long long e_min, int n_bins,
                      unsigned long long* counts, hipStream_t st);
hipError_t launch_dos_direct(const Batch& bt, long long e_min, unsigned long long* counts,
                             hipStream_t st);
hipError_t launch_energy_bound(int N, const int32_t* J, const int32_t* h, long long* out,
                               hipStream_t st);
hipError_t launch_qubo_to_ising(int N, const float* A, const float* b, float* J, float* h,
                                hipStream_t st);
hipError_t launch_qubo_finish(int N, const float* A, const float* b, int S, const uint64_t* found,
                              uint64_t* states_out, float* energies_out, hipStream_t st);
}  // namespace sg

using namespace sg;

namespace {

thread_local std::string g_last_error;

sg_status fail(sg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(SG_EHIP, std::string(#expr ": ") + hipGetErrorString(e_));      \
  } while (0)

// ------------------------------------------------------------------ planning

int ilog2_floor(uint64_t x) { return 63 - __builtin_clzll(x); }

// Low spins per block of a single search: the wider block halves the
// per-block set-up per state once the instance has enough spins for chunks
// of at least 2^8 states per lane; batches and the density of states keep kU.
int search_block(int N) { return N >= 16 ? kUWide : kU; }

struct PlanChunk {
  uint64_t first_mask;
  int n;
  int64_t lanes;
};

// Chunks of [lo, hi) in ascending mask order.  The first chunk has at least
// max(S, 4096) states (it runs with no threshold, so every state is a
// candidate); each next chunk is as large as everything processed before it,
// so that the expected number of candidates per chunk stays near S, until
// the chunk reaches `launch` lanes of 2^nmax states; from then on chunks have
// launch lanes each.  A chunk's free spins n are chosen for `fill` resident
// lanes (n grows once a chunk has more than fill lanes' worth of states), so
// launch >= fill only lets the chunks of n = nmax grow further.  Every chunk
// is [first, first + L 2^n) with first a
// multiple of 2^n, and lanes cover consecutive prefixes.  Ends of the range
// that are not multiples of a block (2^U states) form chunks with n = 0: one
// thread per state, every state a candidate.
std::vector<PlanChunk> plan_chunks(int N, int S, uint64_t lo, uint64_t hi, int64_t fill, int U,
                                   int64_t launch) {
  std::vector<PlanChunk> out;
  const int nmax = std::min(kMaxFree, N);
  if (fill < 1) fill = 1;
  if (launch < fill) launch = fill;
  const int fill_log = ilog2_floor((uint64_t)fill);
  uint64_t target = 4096;
  while (target < (uint64_t)S) target <<= 1;
  const uint64_t big = (uint64_t)launch << nmax;
  const uint64_t blk = (uint64_t)1 << U;
  uint64_t lo_b = (lo + blk - 1) & ~(blk - 1), hi_b = hi & ~(blk - 1);
  if (lo_b >= hi_b) lo_b = hi_b = hi;  // no whole block: one direct chunk
  if (lo < lo_b) out.push_back(PlanChunk{lo, 0, (int64_t)(lo_b - lo)});
  uint64_t cur = lo_b;
  while (cur < hi_b) {
    const uint64_t rem = hi_b - cur;
    PlanChunk c{};
    c.first_mask = cur;
    const uint64_t unit = (uint64_t)1 << nmax;
    if (target >= big && (cur & (unit - 1)) == 0 && rem >= unit) {
      // near the end shrink n rather than the lane count, so that the last
      // chunks still fill the device
      int n = nmax;
      while (n > U && (rem >> n) < (uint64_t)fill) --n;
      c.n = n;
      c.lanes = (int64_t)std::min<uint64_t>((uint64_t)launch, rem >> n);
    } else {
      uint64_t size = std::min<uint64_t>(target, big);
      if (cur != 0) size = std::min<uint64_t>(size, cur & (~cur + 1));
      while (size > rem) size >>= 1;
      const int slog = ilog2_floor(size);
      int n = slog - fill_log;
      n = std::max(n, U);
      n = std::min(n, nmax);
      n = std::min(n, slog);
      c.n = n;
      c.lanes = (int64_t)(size >> n);
    }
    out.push_back(c);
    cur += (uint64_t)c.lanes << c.n;
    target = std::max<uint64_t>(target, 2 * (cur - lo));
  }
  if (hi_b < hi && cur < hi) out.push_back(PlanChunk{cur, 0, (int64_t)(hi - cur)});
  return out;
}

// --------------------------------------------------------------- workspace

// Device buffers of one (device, stream).  Each buffer only grows; growing
// frees the old allocation (hipFree waits for the device), so it never races
// work that earlier calls enqueued.  Once the workspace is pinned (by
// sg_reserve, or by a call made while its stream was capturing a graph), a
// graph may hold its buffers: growing then keeps the old allocation alive
// (retired, released at process exit) instead of freeing it, and a call
// under capture that would need to grow is refused.
struct Workspace {
  int device = -1;
  bool pinned = false;
  bool capturing = false;          // set by ws_get for the call in progress
  std::vector<void*> retired;
  uint32_t* sticky = nullptr;
  Params* P = nullptr;
  size_t nP = 0;
  uint32_t* qtab = nullptr;
  size_t nq = 0;
  uint32_t* table = nullptr;
  size_t ntable = 0;
  uint64_t* cand = nullptr;
  uint32_t* ckey = nullptr;
  uint32_t* skey = nullptr;
  uint64_t* smask = nullptr;
  size_t ncand = 0;
  uint32_t* rkey = nullptr;
  uint64_t* rmask = nullptr;
  uint32_t* tkey = nullptr;
  uint64_t* tmask = nullptr;
  size_t nrec = 0;
  // log Z walk
  double* table64 = nullptr;
  size_t ntable64 = 0;
  // QUBO front end: the Ising instance and the states found before rescoring
  float* qJ = nullptr;
  size_t nqJ = 0;
  float* qh = nullptr;
  size_t nqh = 0;
  uint64_t* qfound = nullptr;
  size_t nqfound = 0;
  float* qenergy = nullptr;
  size_t nqenergy = 0;
  float* lzq = nullptr;        // [B][4][3 * 64] exp(-beta (Q - min Q)) tables
  size_t nlzq = 0;
  double* lzqmin = nullptr;    // [B] min Q
  size_t nlzqmin = 0;
  double* lz_acc = nullptr;
  size_t nlz_acc = 0;
  double* lz_coef = nullptr;
  size_t nlz_coef = 0;
  int64_t fill[2] = {0, 0};      // resident lanes of the walk (fp32, int32)
  int64_t fill_dev[2] = {0, 0};  // the device's values (fill differs only under a test hook)
  int64_t launch[2] = {0, 0};    // lanes per launch of a single search's chunks
  bool tri_all = false;          // test hook: every chunk that can takes the three-field walk
  float margin_scale = 1.0f;     // test hook: factor on the fp32 pruning margin
  int cus = 0;
  // last run
  int64_t last_chunks = 0;
  int64_t last_launches = 0;  // enumeration launches of the last call
  int last_kmax = 0, last_nmax = 0;
  double last_states = 0.0;
  // kernel timing: one event pair per enumeration launch of the last call
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
};

std::atomic<bool> g_timing{false};  // process-wide switch, read by every thread's calls

hipError_t ws_event_pair(Workspace* w, hipEvent_t* a, hipEvent_t* b) {
  while ((int)w->ev.size() < 2 * (w->ev_used + 1)) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    w->ev.push_back(e);
  }
  *a = w->ev[2 * w->ev_used];
  *b = w->ev[2 * w->ev_used + 1];
  ++w->ev_used;
  return hipSuccess;
}

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

// A single search's chunks launch this many times the device's resident
// lanes: the walk's lanes take unequal times (a lane whose blocks fail the
// bound test re-walks them), and with several workgroups per slot the device
// refills a CU as soon as one finishes instead of waiting for the slowest lane
// of a launch (N = 48 dense search: 3.03 s at 8 times the resident lanes,
// 3.86 s at once).
constexpr int64_t kSearchLaunchFills = 8;
// The three-field walk (blocks of kUPk, three per word) takes the chunks of
// at least kTriMinFree free spins that launch at least the resident lanes;
// the others keep the paired walk.  Its exactly walked tail (2 or 4 blocks
// per lane) is a large share at small n, and its coarser fixed point sends
// more blocks to the exact re-walk, which makes lanes uneven where a launch
// cannot balance them: with every chunk of n >= 14 on it, dense searches
// took 46 ms against 36 ms at N = 40 and 348 ms against 331 ms at N = 44;
// with n >= 20 and at least the resident lanes 36, 93 and 304 ms at N = 40,
// 42 and 44 (n >= 20 alone: 38, 109 and 335 ms), and 2.96 s against 4.10 s
// at N = 48 (J ~ N(0, 1)).
constexpr int kTriMinFree = 20;
constexpr uint32_t kCandCapMin = 1u << 22;     // single search
constexpr uint32_t kBatchCandCapMin = 1u << 13;  // per instance of a batch
constexpr uint64_t kBatchCandBudget = 1ull << 24;  // slots over the whole batch

// A call under graph capture that needs a larger buffer: no allocation may be
// enqueued into the graph, and the buffers a replay would use must not move.
constexpr hipError_t kGrowUnderCapture = hipErrorStreamCaptureUnsupported;

template <typename T>
hipError_t grow(Workspace* w, T** p, size_t* have, size_t need) {
  if (*have >= need) return hipSuccess;
  if (w->capturing) return kGrowUnderCapture;
  if (*p) {
    if (w->pinned) {
      w->retired.push_back((void*)*p);  // a captured graph may still use it
    } else {
      hipError_t e = hipFree(*p);
      if (e != hipSuccess) return e;
    }
    *p = nullptr;
    *have = 0;
  }
  hipError_t e = hipMalloc(p, need * sizeof(T));
  if (e == hipSuccess) *have = need;
  return e;
}

// HIP_TRY for workspace growth: a refusal under capture gets its own message.
#define GROW_TRY(expr)                                                                \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ == kGrowUnderCapture)                                                      \
      return fail(SG_EINVAL,                                                          \
                  "the stream is capturing a graph and the workspace is too small for " \
                  "this call: call sg_reserve (or run one call of this shape) first"); \
    if (e_ != hipSuccess)                                                             \
      return fail(SG_ENOMEM, std::string(#expr ": ") + hipGetErrorString(e_));       \
  } while (0)

// The device's compute units and resident lanes (allocates nothing).
sg_status ws_describe(int dev, Workspace* w) {
  w->device = dev;
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SG_EUNSUPPORTED,
                std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  w->cus = prop.multiProcessorCount;
  for (int k = 0; k < 2; ++k) {
    const int occ = enum_occupancy(k == 1);
    w->fill[k] = w->fill_dev[k] = (int64_t)w->cus * std::max(occ, 1) * kEnumBlock;
    w->launch[k] = kSearchLaunchFills * w->fill[k];
  }
  return SG_OK;
}

sg_status ws_create(int dev, Workspace* w) {
  const sg_status v = ws_describe(dev, w);
  if (v != SG_OK) return v;
  HIP_TRY(hipMalloc(&w->sticky, sizeof(uint32_t)));
  HIP_TRY(hipMemset(w->sticky, 0, sizeof(uint32_t)));
  return SG_OK;
}

// The workspace of (current device, stream), created on first use and grown
// to hold B instances with `recs` table records, `cap` candidate slots and S
// record entries each.
sg_status ws_get(hipStream_t st, int B, size_t recs, size_t cap, int S, Workspace** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  const auto key = std::make_pair(dev, st);
  Workspace* w = nullptr;
  auto it = g_ws.find(key);
  if (it != g_ws.end()) {
    w = it->second;
  } else {
    w = new Workspace();
    const sg_status s = ws_create(dev, w);
    if (s != SG_OK) {
      if (w->sticky) (void)hipFree(w->sticky);
      delete w;
      return s;
    }
    g_ws[key] = w;
  }
  // a call enqueued while the stream captures a graph pins the workspace
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
    (void)hipGetLastError();  // not a capture query this stream supports
    cs = hipStreamCaptureStatusNone;
  }
  w->capturing = cs == hipStreamCaptureStatusActive;
  if (w->capturing) w->pinned = true;
  const size_t Bz = (size_t)B;
  GROW_TRY(grow(w, &w->P, &w->nP, Bz));
  GROW_TRY(grow(w, &w->qtab, &w->nq, Bz * kQStride));
  GROW_TRY(grow(w, &w->table, &w->ntable, Bz * recs * kRecWords));
  if (w->ncand < Bz * cap) {
    size_t have_s = w->ncand, have_m = w->ncand, have_c = w->ncand;
    GROW_TRY(grow(w, &w->cand, &w->ncand, Bz * cap));
    GROW_TRY(grow(w, &w->ckey, &have_c, Bz * cap));
    GROW_TRY(grow(w, &w->skey, &have_s, Bz * cap));
    GROW_TRY(grow(w, &w->smask, &have_m, Bz * cap));
  }
  if (w->nrec < Bz * (size_t)S) {
    size_t h1 = w->nrec, h2 = w->nrec, h3 = w->nrec;
    GROW_TRY(grow(w, &w->rkey, &w->nrec, Bz * S));
    GROW_TRY(grow(w, &w->rmask, &h1, Bz * S));
    GROW_TRY(grow(w, &w->tkey, &h2, Bz * S));
    GROW_TRY(grow(w, &w->tmask, &h3, Bz * S));
  }
  *out = w;
  return SG_OK;
}

Batch make_batch(Workspace* w, const void* J, const void* h, const int32_t* Ns, int N0, int ld,
                 int B, int S, int64_t recs, uint32_t cap) {
  Batch bt{};
  bt.J = J;
  bt.h = h;
  bt.Ns = Ns;
  bt.N0 = N0;
  bt.ld = ld;
  bt.B = B;
  bt.S = S;
  bt.P = w->P;
  bt.qtab = w->qtab;
  bt.table = w->table;
  bt.table_recs = recs;
  bt.cand = w->cand;
  bt.ckey = w->ckey;
  bt.skey = w->skey;
  bt.smask = w->smask;
  bt.cap = cap;
  bt.rkey = w->rkey;
  bt.rmask = w->rmask;
  bt.tkey = w->tkey;
  bt.tmask = w->tmask;
  bt.sticky = w->sticky;
  bt.allow_f32_walk = 1;
  bt.margin_scale = w->margin_scale;
  return bt;
}

// Records of the concatenated per-block tables for n = U .. ncap.
size_t table_records(int ncap) { return ((size_t)1 << (ncap - kU + 1)) - 1; }
size_t lz_table_records(int ncap, int U) { return ((size_t)1 << (ncap - U + 1)) - 1; }

// ------------------------------------------------------------------ search

sg_status validate(int N, const void* J, const void* h, int S, uint64_t lo, uint64_t hi,
                   const void* so, const void* eo) {
  if (N < 1 || N > SG_MAX_N) return fail(SG_EINVAL, "N must be in [1, SG_MAX_N]");
  if (!J || !h || !so || !eo) return fail(SG_EINVAL, "null pointer argument");
  const uint64_t full = (uint64_t)1 << N;
  if (!(lo < hi) || hi > full) return fail(SG_EINVAL, "need mask_lo < mask_hi <= 2^N");
  if ((lo % 64) != 0 || ((hi % 64) != 0 && hi != full))
    return fail(SG_EINVAL, "mask_lo and mask_hi must be multiples of 64 (or mask_hi = 2^N)");
  if (S < 1 || S > SG_MAX_S) return fail(SG_EINVAL, "S must be in [1, SG_MAX_S]");
  if ((uint64_t)S > hi - lo) return fail(SG_EINVAL, "S exceeds the number of states searched");
  return SG_OK;
}

// split: test the walk's bound per 64-step sub-block (batched searches)
hipError_t enum_timed(Workspace* w, bool isint, int U, bool split, const Batch& bt,
                      const Chunk& ch, int ninst, hipStream_t st) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (g_timing) {
    hipError_t r = ws_event_pair(w, &e0, &e1);
    if (r != hipSuccess) return r;
    r = hipEventRecord(e0, st);
    if (r != hipSuccess) return r;
  }
  hipError_t r = launch_enum(isint, U, split, bt, ch, ninst, st);
  if (r != hipSuccess) return r;
  ++w->last_launches;
  if (g_timing) r = hipEventRecord(e1, st);
  return r;
}

// Enqueue the search of [lo, hi) on workspace w, whose buffers hold `recs`
// table records, `cap` candidate slots and S record entries.
sg_status search_on(Workspace* w, bool isint, int N, const void* J, const void* h, int S,
                    uint64_t lo, uint64_t hi, size_t recs, uint32_t cap, uint64_t* states_out,
                    void* energies_out, hipStream_t st) {
  const int U = search_block(N);
  const int ncap = std::min(kMaxFree, std::max(N, U));
  Batch bt = make_batch(w, J, h, nullptr, N, N, 1, S, (int64_t)recs, cap);
  // chunks of n >= kUPk + 2 free spins walk blocks of kUPk (paired, fp32
  // walks; three at a time from n >= kUPk + kTriMinM); their tables follow
  // the records of U = kUWide
  bt.tri = 1;
  const bool use10 = U == kUWide && ncap >= kUPk + 2;
  bt.table_base10w = (int64_t)(((size_t)1 << (ncap - kUWide + 1)) - 1) * kRecWords;
  if (use10 && (size_t)bt.table_base10w + (((size_t)1 << (ncap - kUPk + 1)) - 1) *
                                               (size_t)rec_words(kUPk) >
                   recs * (size_t)kRecWords)
    return fail(SG_EUNSUPPORTED, "table buffer too small for the blocks of 10");

  HIP_TRY(launch_prep(isint, bt, st));
  const int score_grid = std::max(1, w->cus) * 4;
  int kmax = 0, nmaxu = 0;
  w->ev_used = 0;
  w->last_launches = 0;
  if (N >= U) HIP_TRY(launch_tables(isint, U, bt, ncap, true, st));
  if (use10) HIP_TRY(launch_tables(isint, kUPk, bt, ncap, true, st));
  // chunks planned for the lanes of a launch (free spins included), not the
  // resident lanes: more, shorter lanes per chunk let the device balance them
  // (dense searches at N = 40, 42, 44: 23, 70 and 255 ms against 33, 91 and
  // 299 ms planned for the resident lanes; N = 48 unchanged)
  const int64_t launch = w->launch[isint ? 1 : 0];
  const std::vector<PlanChunk> plan = plan_chunks(N, S, lo, hi, launch, U, launch);
  double states = 0.0;
  for (const PlanChunk& pc : plan) {
    if (pc.n == 0) {
      // a range end shorter than a block: one thread per state
      HIP_TRY(launch_direct(bt, pc.first_mask, pc.first_mask + (uint64_t)pc.lanes, st));
      HIP_TRY(launch_score(isint, bt, 0, score_grid, N, 0, st));
      HIP_TRY(launch_merge(bt, 0, 0, true, st));
      states += (double)pc.lanes;
      continue;
    }
    Chunk ch{};
    ch.first_mask = pc.first_mask;
    ch.prefix_base = pc.first_mask >> pc.n;
    ch.lanes = pc.lanes;
    ch.n = pc.n;
    const int Uc = use10 && pc.n >= kUPk + 2 ? kUPk : U;
    ch.table_offset = (1 << (pc.n - Uc)) - 1;
    ch.table_offset8 = (1 << (pc.n - U)) - 1;
    ch.tri = Uc == kUPk && pc.n >= kUPk + kTriMinM &&
             (w->tri_all || (pc.n >= kTriMinFree && pc.lanes >= w->fill_dev[isint ? 1 : 0]));
    // a chunk with more states than candidate slots may overflow: it gets
    // up to kRetries repeated passes, each run only if the last overflowed
    const uint64_t cstates = (uint64_t)pc.lanes << pc.n;
    const int passes = cstates > (uint64_t)cap ? 1 + kRetries : 1;
    for (int r = 0; r < passes; ++r) {
      ch.retry = r;
      HIP_TRY(enum_timed(w, isint, Uc, false, bt, ch, 1, st));
      HIP_TRY(launch_score(isint, bt, 0, score_grid, N, r, st));
      HIP_TRY(launch_merge(bt, 0, r, r == passes - 1, st));
    }
    states += (double)cstates;
    kmax = std::max(kmax, N - pc.n);
    nmaxu = std::max(nmaxu, pc.n);
  }
  const int64_t nchunks = (int64_t)plan.size();
  w->last_states = states;
  HIP_TRY(launch_finalize(isint, bt, states_out, energies_out, st));
  w->last_chunks = nchunks;
  w->last_kmax = kmax;
  w->last_nmax = nmaxu;
  return SG_OK;
}

sg_status run_search(bool isint, int N, const void* J, const void* h, int S, uint64_t lo,
                     uint64_t hi, uint64_t* states_out, void* energies_out, void* stream) {
  g_last_error.clear();
  sg_status v = validate(N, J, h, S, lo, hi, states_out, energies_out);
  if (v != SG_OK) return v;
  hipStream_t st = (hipStream_t)stream;
  uint32_t cap = kCandCapMin;
  while (cap < 8u * (uint32_t)S) cap <<= 1;
  const size_t recs = table_records(kMaxFree);  // blocks of kU outnumber those of kUWide
  Workspace* w = nullptr;
  v = ws_get(st, 1, recs, cap, S, &w);
  if (v != SG_OK) return v;
  return search_on(w, isint, N, J, h, S, lo, hi, recs, cap, states_out, energies_out, st);
}

// Level geometry of the batched search: n = log2(level size) - shift free
// spins per lane (clamped), i.e. 2^shift lanes per instance.  The default is
// 2^12 lanes per instance, the fastest geometry measured on 4096 instances of
// 16..32 spins (fewer free spins per lane spend more of each lane on its
// set-up; more leave too few lanes once the smaller instances have finished),
// and more when B is too small for B 2^shift to reach four times the
// device's resident lanes (256 instances of 28 spins: 2^13 lanes each, 5%
// faster than 2^12).  The tuner (sg_tune_batched_f32) may pick another shift per
// (device, B, N_max, S).
constexpr int kShiftFloor = 12;
constexpr int kShiftSpan = 3;  // the tuner tries default - 3 .. default + 3
std::map<std::tuple<int, int, int, int>, int> g_shift;  // (device, B, N_max, S) -> shift

int default_shift(int B, int64_t fill) {
  int shift = 0;
  while (shift < 40 && ((int64_t)B << shift) < 4 * fill) ++shift;
  return std::max(shift, kShiftFloor);
}

int batch_shift(int B, int Nmax, int S, int64_t fill) {
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_shift.find(std::make_tuple(dev, B, Nmax, S));
    if (it != g_shift.end()) return it->second;
  }
  return default_shift(B, fill);
}

// Chunk levels of a batched search.  Level 0 is [0, first) with
// first = max(S, 4096) rounded up to a power of two: every state of it is a
// candidate (at most half the 8192 or more slots an instance has), and one
// such level replaces the five smallest doubling levels, whose launches and
// merges cost far more than their states; level j >= 1 is
// [first 2^(j-1), first 2^j),
// so every level is as large as everything before it and brings about S
// candidates.  All instances with states in a level run it in the same launch,
// with the same geometry: n = clamp(log2(size) - shift, kU, kBatchFreeCap) free spins per
// lane.
constexpr uint64_t kBatchLevel0 = 4096;  // smallest level 0 (<= half of any instance's slots)
struct Level {
  uint64_t first;
  int n;
  int64_t lanes;
};

std::vector<Level> batch_levels(int Nmax, int S, int shift) {
  std::vector<Level> out;
  uint64_t size0 = kBatchLevel0;
  while (size0 < (uint64_t)S) size0 <<= 1;
  const uint64_t full = (uint64_t)1 << Nmax;
  uint64_t first = 0, size = size0;
  while (first < full) {
    const int a = ilog2_floor(size);
    int n = std::max(kU, std::min(kBatchFreeCap, a - shift));
    n = std::min(n, a);
    out.push_back(Level{first, n, (int64_t)(size >> n)});
    first += size;
    size = first;
  }
  return out;
}

// Enqueue the batched search over bt (levels of batch_levels) and its
// finalize into states_out / energies_out.
sg_status batch_search(Workspace* w, bool isint, const Batch& bt0, int Nmax, int ncap,
                       uint64_t* states_out, void* energies_out, hipStream_t st) {
  // levels whose lanes have n >= kUPk + 2 free spins walk blocks of kUPk,
  // those of n >= kUWide blocks of kUWide, the others (n = kU) blocks of kU:
  // the one record of n = kU comes first, then the records of kUWide for
  // n = kUWide .. ncap, then those of kUPk
  Batch bt = bt0;
  bt.table_base8 = (int64_t)table_records(kU);
  // levels of n >= kUPk + 2 walk blocks of kUPk (paired, fp32 walks), from
  // tables that follow those of kUWide in each instance's region
  const bool use10 = ncap >= kUPk + 2;
  bt.table_base10w =
      (bt.table_base8 + (int64_t)(((size_t)1 << (ncap - kUWide + 1)) - 1)) * kRecWords;
  if (use10 && (size_t)bt.table_base10w + (((size_t)1 << (ncap - kUPk + 1)) - 1) *
                                               (size_t)rec_words(kUPk) >
                   (size_t)bt.table_recs * kRecWords)
    return fail(SG_EUNSUPPORTED, "table buffer too small for the blocks of 10");
  HIP_TRY(launch_prep(isint, bt, st));
  HIP_TRY(launch_tables(isint, kU, bt, kU, false, st));
  if (ncap >= kUWide) HIP_TRY(launch_tables(isint, kUWide, bt, ncap, true, st));
  if (use10) HIP_TRY(launch_tables(isint, kUPk, bt, ncap, true, st));
  const std::vector<Level> levels =
      batch_levels(Nmax, bt.S, batch_shift(bt.B, Nmax, bt.S, w->fill[isint ? 1 : 0]));
  w->ev_used = 0;
  w->last_launches = 0;
  double states = 0.0;
  int nmaxu = 0;
  for (const Level& L : levels) {
    Chunk ch{};
    ch.first_mask = L.first;
    ch.prefix_base = L.first >> L.n;
    ch.lanes = L.lanes;
    ch.n = L.n;
    const int U = use10 && L.n >= kUPk + 2 ? kUPk : L.n >= kUWide ? kUWide : kU;
    ch.table_offset = U == kUPk ? (1 << (L.n - kUPk)) - 1
                                : (U == kUWide ? (int)bt.table_base8 : 0) + (1 << (L.n - U)) - 1;
    ch.table_offset8 = (int)bt.table_base8 + (1 << (L.n - kUWide)) - 1;
    const uint64_t lstates = (uint64_t)L.lanes << L.n;
    const int passes = lstates > (uint64_t)bt.cap ? 1 + kRetries : 1;
    for (int r = 0; r < passes; ++r) {
      ch.retry = r;
      HIP_TRY(enum_timed(w, isint, U, true, bt, ch, bt.B, st));
      HIP_TRY(launch_merge_batched(isint, bt, L.first, r, r == passes - 1, st));
    }
    states += (double)lstates;
    nmaxu = std::max(nmaxu, L.n);
  }
  HIP_TRY(launch_finalize(isint, bt, states_out, energies_out, st));
  w->last_chunks = (int64_t)levels.size();
  w->last_kmax = Nmax - nmaxu;
  w->last_nmax = nmaxu;
  w->last_states = states;
  return SG_OK;
}

// Candidate slots per instance of a batch: at least 8192 and 4 S, more for
// small batches (up to kBatchCandBudget slots in all, 20 bytes each).
uint32_t batch_cap(int B, int S) {
  uint32_t cap = kBatchCandCapMin;
  while (cap < 2u * 4096u || cap < 4u * (uint32_t)S) cap <<= 1;
  while (cap < (1u << 20) && (uint64_t)(2u * cap) * (uint64_t)B <= kBatchCandBudget) cap <<= 1;
  return cap;
}

sg_status run_batched(bool isint, int B, const int32_t* Ns, int Nmax, const void* J,
                      const void* h, int S, uint64_t* states_out, void* energies_out,
                      void* stream) {
  g_last_error.clear();
  if (B < 1) return fail(SG_EINVAL, "B must be >= 1");
  if (Nmax < kU || Nmax > kMaxNBatched) return fail(SG_EINVAL, "N_max must be in [7, 40]");
  if (S < 1 || S > SG_MAX_S_BATCHED) return fail(SG_EINVAL, "S must be in [1, SG_MAX_S_BATCHED]");
  if (!Ns || !J || !h || !states_out || !energies_out)
    return fail(SG_EINVAL, "null pointer argument");
  hipStream_t st = (hipStream_t)stream;
  const uint32_t cap = batch_cap(B, S);
  const int ncap = std::min(kBatchFreeCap, Nmax);
  const size_t recs = table_records(ncap);
  Workspace* w = nullptr;
  sg_status v = ws_get(st, B, recs, cap, S, &w);
  if (v != SG_OK) return v;
  const Batch bt = make_batch(w, J, h, Ns, 0, Nmax, B, S, (int64_t)recs, cap);
  return batch_search(w, isint, bt, Nmax, ncap, states_out, energies_out, st);
}

// ------------------------------------------------------------------ log Z

sg_status lz_validate(int B, int N, const void* J, const void* h, int nb, const void* beta) {
  if (B < 1) return fail(SG_EINVAL, "B must be >= 1");
  if (N < kU || N > 40) return fail(SG_EINVAL, "N must be in [7, 40]");
  if (nb < 1 || nb > kMaxBeta) return fail(SG_EINVAL, "n_beta must be in [1, 4]");
  if (!J || !h || !beta) return fail(SG_EINVAL, "null pointer argument");
  return SG_OK;
}

sg_status lz_buffers(Workspace* w, int B, int N) {
  const size_t Bz = (size_t)B;
  const size_t stride = std::max<size_t>(kMaxBeta, (size_t)N * N + N);
  // records of U = kLzU outnumber (and outsize) those of U = kLzUF
  GROW_TRY(grow(w, &w->table64, &w->ntable64,
                Bz * lz_table_records(std::min(kLzFree, N), kLzU) * (2 + kLzUF)));
  GROW_TRY(grow(w, &w->lzq, &w->nlzq, Bz * kMaxBeta * kLzQStride));
  GROW_TRY(grow(w, &w->lzqmin, &w->nlzqmin, Bz));
  GROW_TRY(grow(w, &w->lz_acc, &w->nlz_acc, Bz * stride));
  GROW_TRY(grow(w, &w->lz_coef, &w->nlz_coef, Bz * 2 * kMaxBeta));
  return SG_OK;
}

// The walk's geometry for `fill` resident lanes; coef, acc and sticky are
// left for the caller to point at its buffers.
LzArgs lz_geometry(int64_t fill, int B, int N, int nb, int S, const float* h, const float* beta,
                   const float* e0, int mode) {
  LzArgs a{};
  a.B = B;
  a.N = N;
  // low spins per block (record): the larger blocks whenever the instance
  // has that many spins (the gradient walk's records hold four sub-blocks
  // of kLzU; the partition sums of four beta keep records of 8, which fit
  // their registers)
  a.U = (mode == 0 && N >= kLzUW && nb <= 3) ? kLzUW : N >= kLzUF ? kLzUF : kLzU;
  // free spins per lane: at most kLzFree, fewer when the batch alone would
  // not give every resident lane of the device a prefix
  a.n = std::min(kLzFree, N);
  while (a.n > a.U && (int64_t)B * ((int64_t)1 << (N - a.n)) < fill) --a.n;
  a.nb = nb;
  a.S = S;
  a.lanes = (int64_t)1 << (N - a.n);
  a.table_recs = (int64_t)lz_table_records(a.n, a.U);
  a.table_offset = (1 << (a.n - a.U)) - 1;
  a.h_in = h;
  a.beta = beta;
  a.e0 = e0;
  a.acc_stride = mode == 0 ? kMaxBeta : N * N + N;
  return a;
}

LzArgs lz_args(Workspace* w, int B, int N, int nb, int S, const float* h, const float* beta,
               const float* e0, int mode) {
  LzArgs a = lz_geometry(w->fill[0], B, N, nb, S, h, beta, e0, mode);
  a.coef = w->lz_coef;
  a.acc = w->lz_acc;
  a.sticky = w->sticky;
  return a;
}

// Resident lanes of the fp32 walk on device dev, for calls that have no
// workspace (queried once per device; allocates no device memory).
std::map<int, int64_t> g_dev_fill;

sg_status device_fill(int dev, int64_t* fill) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev_fill.find(dev);
    if (it != g_dev_fill.end()) {
      *fill = it->second;
      return SG_OK;
    }
  }
  Workspace probe;
  const sg_status v = ws_describe(dev, &probe);
  if (v != SG_OK) return v;
  std::lock_guard<std::mutex> lk(g_mu);
  g_dev_fill[dev] = probe.fill[0];
  *fill = probe.fill[0];
  return SG_OK;
}

Workspace* ws_find(hipStream_t st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find(std::make_pair(dev, st));
  return it == g_ws.end() ? nullptr : it->second;
}

sg_status status_of_bits(uint32_t bits) {
  if (bits & kErrInval)
    return fail(SG_EINVAL,
                "device-side argument check: N_b outside [6, N_max], S > 2^N_b, or a beta not > 0");
  if (bits & kErrNonFinite) return fail(SG_ENONFINITE, "NaN or Inf in J or h");
  if (bits & kErrOverflow)
    return fail(SG_EOVERFLOW, "integer instance too large: sum|J| + sum|h| must be < 2^28");
  if (bits & kErrCapacity) return fail(SG_ECAPACITY, "candidate buffer overflowed");
  if (bits & kErrDrift) return fail(SG_EDRIFT, "fp32 drift exceeded its bound");
  return SG_OK;
}

}  // namespace

extern "C" {

sg_status sg_low_spectrum_f32(int N, const float* J, const float* h, int S, uint64_t* states_out,
                              float* energies_out, void* stream) {
  if (N < 1 || N > SG_MAX_N) return fail(SG_EINVAL, "N must be in [1, SG_MAX_N]");
  return run_search(false, N, J, h, S, 0, (uint64_t)1 << N, states_out, energies_out, stream);
}

sg_status sg_low_spectrum_i32(int N, const int32_t* J, const int32_t* h, int S,
                              uint64_t* states_out, int32_t* energies_out, void* stream) {
  if (N < 1 || N > SG_MAX_N) return fail(SG_EINVAL, "N must be in [1, SG_MAX_N]");
  return run_search(true, N, J, h, S, 0, (uint64_t)1 << N, states_out, energies_out, stream);
}

sg_status sg_low_spectrum_range_f32(int N, const float* J, const float* h, int S, uint64_t lo,
                                    uint64_t hi, uint64_t* states_out, float* energies_out,
                                    void* stream) {
  return run_search(false, N, J, h, S, lo, hi, states_out, energies_out, stream);
}

sg_status sg_low_spectrum_range_i32(int N, const int32_t* J, const int32_t* h, int S,
                                    uint64_t lo, uint64_t hi, uint64_t* states_out,
                                    int32_t* energies_out, void* stream) {
  return run_search(true, N, J, h, S, lo, hi, states_out, energies_out, stream);
}

sg_status sg_low_spectrum_batched_f32(int B, const int32_t* N_dev, int N_max, const float* J,
                                      const float* h, int S, uint64_t* states_out,
                                      float* energies_out, void* stream) {
  return run_batched(false, B, N_dev, N_max, J, h, S, states_out, energies_out, stream);
}

sg_status sg_low_spectrum_batched_i32(int B, const int32_t* N_dev, int N_max, const int32_t* J,
                                      const int32_t* h, int S, uint64_t* states_out,
                                      int32_t* energies_out, void* stream) {
  return run_batched(true, B, N_dev, N_max, J, h, S, states_out, energies_out, stream);
}

sg_status sg_logz_forward_f32(int B, int N, const float* J, const float* h, int n_beta,
                              const float* beta, int S, double* logz_out, float* e0_out,
                              uint64_t* states_out, float* energies_out, void* stream) {
  g_last_error.clear();
  sg_status v = lz_validate(B, N, J, h, n_beta, beta);
  if (v != SG_OK) return v;
  if (!logz_out || !e0_out || !states_out || !energies_out)
    return fail(SG_EINVAL, "null pointer argument");
  if (S < 1 || S > SG_MAX_S_BATCHED || (uint64_t)S > ((uint64_t)1 << N))
    return fail(SG_EINVAL, "S must be in [1, min(SG_MAX_S_BATCHED, 2^N)]");
  hipStream_t st = (hipStream_t)stream;
  const uint32_t cap = batch_cap(B, S);
  const int ncap = std::min(kBatchFreeCap, N);
  const size_t recs = table_records(ncap);
  Workspace* w = nullptr;
  v = ws_get(st, B, recs, cap, S, &w);
  if (v != SG_OK) return v;
  v = lz_buffers(w, B, N);
  if (v != SG_OK) return v;
  // 1. low spectrum of every instance (E0 and the S lowest states)
  const Batch bt = make_batch(w, J, h, nullptr, N, N, B, S, (int64_t)recs, cap);
  v = batch_search(w, false, bt, N, ncap, states_out, energies_out, st);
  if (v != SG_OK) return v;
  // 2. partition sums shifted by E0
  const LzArgs a = lz_args(w, B, N, n_beta, S, h, beta, e0_out, 0);
  Batch b64 = bt;
  b64.table_recs = a.table_recs;
  HIP_TRY(launch_tables64(b64, a.n, a.U, w->table64, st));
  HIP_TRY(launch_lz_prep(0, a, J, w->lzq, w->lzqmin, energies_out, e0_out, nullptr, nullptr, st));
  HIP_TRY(launch_logz(0, a, J, h, w->table64, w->lzq, w->lzqmin, st));
  HIP_TRY(launch_lz_final(0, a, logz_out, nullptr, nullptr, st));
  return SG_OK;
}

sg_status sg_logz_backward_f32(int B, int N, const float* J, const float* h, int n_beta,
                               const float* beta, const float* e0, const double* logz,
                               const double* grad_logz, float* grad_J, float* grad_h,
                               void* stream) {
  g_last_error.clear();
  sg_status v = lz_validate(B, N, J, h, n_beta, beta);
  if (v != SG_OK) return v;
  if (!e0 || !logz || !grad_logz || !grad_J || !grad_h)
    return fail(SG_EINVAL, "null pointer argument");
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = nullptr;
  v = ws_get(st, B, 1, 1, 1, &w);
  if (v != SG_OK) return v;
  v = lz_buffers(w, B, N);
  if (v != SG_OK) return v;
  const LzArgs a = lz_args(w, B, N, n_beta, 1, h, beta, e0, 1);
  Batch b64 = make_batch(w, J, h, nullptr, N, N, B, 1, a.table_recs, 1);
  HIP_TRY(launch_tables64(b64, a.n, a.U, w->table64, st));
  HIP_TRY(launch_lz_prep(1, a, J, w->lzq, w->lzqmin, nullptr, nullptr, logz, grad_logz, st));
  HIP_TRY(launch_logz(1, a, J, h, w->table64, w->lzq, w->lzqmin, st));
  HIP_TRY(launch_lz_final(1, a, nullptr, grad_J, grad_h, st));
  return SG_OK;
}

static_assert(SG_LOGZ_SCRATCH_BYTES == kLzScratchBytes, "scratch size differs from the header");

sg_status sg_logz_backward_noalloc_f32(int B, int N, const float* J, const float* h, int n_beta,
                                       const float* beta, const float* e0, const double* logz,
                                       const double* grad_logz, float* grad_J, float* grad_h,
                                       void* stream) {
  g_last_error.clear();
  sg_status v = lz_validate(B, N, J, h, n_beta, beta);
  if (v != SG_OK) return v;
  if (!e0 || !logz || !grad_logz || !grad_J || !grad_h)
    return fail(SG_EINVAL, "null pointer argument");
  hipStream_t st = (hipStream_t)stream;
  // the decomposition of sg_logz_backward_f32 on this stream
  int64_t fill = 0;
  if (Workspace* w = ws_find(st)) {
    fill = w->fill[0];
  } else {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    v = device_fill(dev, &fill);
    if (v != SG_OK) return v;
  }
  LzArgs a = lz_geometry(fill, B, N, n_beta, 1, h, beta, e0, 1);
  // scratch layout: the error word, then each buffer at a 256-byte boundary
  const size_t Bz = (size_t)B;
  size_t used = 256;
  auto take = [&used](size_t bytes) {
    const size_t at = used;
    used += (bytes + 255) & ~(size_t)255;
    return at;
  };
  const size_t o_tab = take(Bz * (size_t)a.table_recs * (2 + a.U) * sizeof(double));
  const size_t o_q = take(Bz * kMaxBeta * (size_t)lz_q_stride(a.U) * sizeof(float));
  const size_t o_qmin = take(Bz * sizeof(double));
  const size_t o_acc = take(Bz * (size_t)a.acc_stride * sizeof(double));
  const size_t o_coef = take(Bz * 2 * kMaxBeta * sizeof(double));
  if (used > kLzScratchBytes)
    return fail(SG_EINVAL, "B = " + std::to_string(B) + ", N = " + std::to_string(N) +
                               " needs " + std::to_string(used) +
                               " bytes of device scratch, more than the SG_LOGZ_SCRATCH_BYTES = " +
                               std::to_string(kLzScratchBytes) +
                               " this entry point holds (sg_logz_backward_f32 has no such limit)");
  void* base = nullptr;
  bool fresh = false;
  HIP_TRY(lz_scratch(&base, &fresh));
  char* sp = (char*)base;
  uint32_t* err = (uint32_t*)sp;
  if (fresh) HIP_TRY(launch_clear_word(err, st));
  double* tab = (double*)(sp + o_tab);
  float* lzq = (float*)(sp + o_q);
  double* lzqmin = (double*)(sp + o_qmin);
  a.acc = (double*)(sp + o_acc);  // cleared by the prep kernel
  a.coef = (double*)(sp + o_coef);
  a.sticky = err;
  Batch b64{};
  b64.J = J;
  b64.h = h;
  b64.Ns = nullptr;
  b64.N0 = N;
  b64.ld = N;
  b64.B = B;
  b64.table_recs = a.table_recs;
  HIP_TRY(launch_tables64(b64, a.n, a.U, tab, st));
  HIP_TRY(launch_lz_prep(1, a, J, lzq, lzqmin, nullptr, nullptr, logz, grad_logz, st));
  HIP_TRY(launch_logz(1, a, J, h, tab, lzq, lzqmin, st));
  HIP_TRY(launch_lz_final(1, a, nullptr, grad_J, grad_h, st));
  return SG_OK;
}

sg_status sg_reserve(int B_max, int N_max, int S_max, void* stream) {
  g_last_error.clear();
  if (B_max < 1) return fail(SG_EINVAL, "B_max must be >= 1");
  if (N_max < 1 || N_max > SG_MAX_N) return fail(SG_EINVAL, "N_max must be in [1, SG_MAX_N]");
  if (S_max < 1 || S_max > SG_MAX_S) return fail(SG_EINVAL, "S_max must be in [1, SG_MAX_S]");
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = nullptr;
  // single-instance search
  uint32_t cap = kCandCapMin;
  while (cap < 8u * (uint32_t)S_max) cap <<= 1;
  sg_status v = ws_get(st, 1, table_records(kMaxFree), cap, S_max, &w);
  if (v != SG_OK) return v;
  w->pinned = true;  // a graph captured from here on may hold these buffers
  // batched search and log Z
  if (N_max >= kU && N_max <= kMaxNBatched && S_max <= SG_MAX_S_BATCHED) {
    // the per-instance slots grow as B shrinks: size for the largest B * cap
    uint64_t slots = 0;
    for (int b = 1; b <= B_max; ++b) slots = std::max(slots, (uint64_t)b * batch_cap(b, S_max));
    const size_t cap_b = (size_t)((slots + B_max - 1) / B_max);
    v = ws_get(st, B_max, table_records(std::min(kBatchFreeCap, N_max)), cap_b, S_max, &w);
    if (v != SG_OK) return v;
    v = lz_buffers(w, B_max, N_max);
    if (v != SG_OK) return v;
  }
  return SG_OK;
}

sg_status sg_energy_bound_i32(int N, const int32_t* J, const int32_t* h, long long* bound_out,
                              void* stream) {
  g_last_error.clear();
  if (N < 1 || N > SG_MAX_N) return fail(SG_EINVAL, "N must be in [1, SG_MAX_N]");
  if (!J || !h || !bound_out) return fail(SG_EINVAL, "null pointer argument");
  HIP_TRY(launch_energy_bound(N, J, h, bound_out, (hipStream_t)stream));
  return SG_OK;
}

sg_status sg_density_of_states_i32(int N, const int32_t* J, const int32_t* h, long long e_min,
                                   int n_bins, unsigned long long* counts_out, void* stream) {
  g_last_error.clear();
  if (N < 1 || N > SG_MAX_N) return fail(SG_EINVAL, "N must be in [1, SG_MAX_N]");
  if (n_bins < 1 || n_bins > SG_MAX_DOS_BINS)
    return fail(SG_EINVAL, "n_bins must be in [1, SG_MAX_DOS_BINS]");
  if (!J || !h || !counts_out) return fail(SG_EINVAL, "null pointer argument");
  hipStream_t st = (hipStream_t)stream;
  const size_t recs = table_records(kMaxFree);
  Workspace* w = nullptr;
  sg_status v = ws_get(st, 1, recs, 1, 1, &w);
  if (v != SG_OK) return v;
  Batch bt = make_batch(w, J, h, nullptr, N, N, 1, 1, (int64_t)recs, 1);
  bt.allow_f32_walk = 0;  // the histogram walk reads integer tables
  HIP_TRY(launch_prep(true, bt, st));
  HIP_TRY(launch_dos_prologue(bt, e_min, n_bins, counts_out, st));
  w->ev_used = 0;
  w->last_launches = 0;
  double states = 0.0;
  if (N < kU) {
    HIP_TRY(launch_dos_direct(bt, e_min, counts_out, st));
    states = (double)((uint64_t)1 << N);
  } else {
    // n free spins per lane: at most kMaxFree, fewer while the prefixes would
    // not give every resident lane one; launches of at most `fill` lanes
    const int64_t fill = w->fill[1];
    int n = std::min(kMaxFree, N);
    while (n > kU && ((int64_t)1 << (N - n)) < fill) --n;
    HIP_TRY(launch_tables(true, kU, bt, n, false, st));
    const uint64_t prefixes = (uint64_t)1 << (N - n);
    for (uint64_t base = 0; base < prefixes; base += (uint64_t)fill) {
      Chunk ch{};
      ch.prefix_base = base;
      ch.first_mask = base << n;
      ch.lanes = (int64_t)std::min<uint64_t>((uint64_t)fill, prefixes - base);
      ch.n = n;
      ch.table_offset = (1 << (n - kU)) - 1;
      HIP_TRY(launch_dos(bt, ch, e_min, n_bins, counts_out, st));
      ++w->last_launches;
      states += (double)ch.lanes * (double)((uint64_t)1 << n);
    }
  }
  w->last_chunks = w->last_launches;
  w->last_states = states;
  return SG_OK;
}

sg_status sg_tune_batched_f32(int B, const int32_t* N_dev, int N_max, const float* J,
                              const float* h, int S, int* shift_out, void* stream) {
  g_last_error.clear();
  if (!shift_out) return fail(SG_EINVAL, "null pointer argument");
  if (B < 1 || S < 1) return fail(SG_EINVAL, "B and S must be >= 1");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = nullptr;
  sg_status v = ws_get(st, B, 1, 1, 1, &w);
  if (v != SG_OK) return v;
  const auto key = std::make_tuple(dev, B, N_max, S);
  const int centre = default_shift(B, w->fill[0]);
  const int lo_shift = std::max(0, centre - kShiftSpan), hi_shift = centre + kShiftSpan;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_shift.erase(key);
  }
  uint64_t* tm = nullptr;
  float* te = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMalloc(&tm, sizeof(uint64_t) * (size_t)B * S) != hipSuccess ||
      hipMalloc(&te, sizeof(float) * (size_t)B * S) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    v = fail(SG_ENOMEM, "tuner scratch allocation failed");
  float best_ms = 0.0f;
  int best = centre;
  for (int shift = lo_shift; shift <= hi_shift && v == SG_OK; ++shift) {
    {
      std::lock_guard<std::mutex> lk(g_mu);
      g_shift[key] = shift;
    }
    v = sg_low_spectrum_batched_f32(B, N_dev, N_max, J, h, S, tm, te, stream);  // warm-up
    float ms = 0.0f;
    for (int r = 0; r < 2 && v == SG_OK; ++r) {
      if (hipEventRecord(e0, st) != hipSuccess) v = fail(SG_EHIP, "hipEventRecord");
      if (v == SG_OK) v = sg_low_spectrum_batched_f32(B, N_dev, N_max, J, h, S, tm, te, stream);
      if (v == SG_OK && hipEventRecord(e1, st) != hipSuccess) v = fail(SG_EHIP, "hipEventRecord");
      if (v == SG_OK && hipEventSynchronize(e1) != hipSuccess) v = fail(SG_EHIP, "sync");
      float t = 0.0f;
      if (v == SG_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) v = fail(SG_EHIP, "time");
      ms += t;
    }
    if (v == SG_OK) v = sg_get_error(stream);
    if (v == SG_OK && (shift == lo_shift || ms < best_ms)) {
      best_ms = ms;
      best = shift;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (v == SG_OK) g_shift[key] = best;
    else g_shift.erase(key);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (tm) (void)hipFree(tm);
  if (te) (void)hipFree(te);
  if (v != SG_OK) return v;
  *shift_out = best;
  return SG_OK;
}

sg_status sg_low_spectrum_qubo_f32(int N, const float* A, const float* b, int S,
                                   uint64_t* states_out, float* energies_out, void* stream) {
  g_last_error.clear();
  if (N < 1 || N > SG_MAX_N) return fail(SG_EINVAL, "N must be in [1, SG_MAX_N]");
  if (S < 1 || S > kQuboSortCap || (N < 63 && (uint64_t)S > ((uint64_t)1 << N)))
    return fail(SG_EINVAL, "S must be in [1, min(SG_MAX_S_BATCHED, 2^N)]");
  if (!A || !b || !states_out || !energies_out) return fail(SG_EINVAL, "null pointer argument");
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = nullptr;
  sg_status v = ws_get(st, 1, 1, 1, 1, &w);
  if (v != SG_OK) return v;
  GROW_TRY(grow(w, &w->qJ, &w->nqJ, (size_t)N * N));
  GROW_TRY(grow(w, &w->qh, &w->nqh, (size_t)N));
  GROW_TRY(grow(w, &w->qfound, &w->nqfound, (size_t)S));
  GROW_TRY(grow(w, &w->qenergy, &w->nqenergy, (size_t)S));
  HIP_TRY(launch_qubo_to_ising(N, A, b, w->qJ, w->qh, st));
  v = run_search(false, N, w->qJ, w->qh, S, 0, (uint64_t)1 << N, w->qfound, w->qenergy, stream);
  if (v != SG_OK) return v;
  HIP_TRY(launch_qubo_finish(N, A, b, S, w->qfound, states_out, energies_out, st));
  return SG_OK;
}

sg_status sg_get_error(void* stream) {
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(st));
  uint32_t bits = 0;
  if (Workspace* w = ws_find(st)) {
    HIP_TRY(hipMemcpy(&bits, w->sticky, sizeof(bits), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(w->sticky, 0, sizeof(uint32_t)));
  }
  // the error word of the device's static scratch (allocation-free calls)
  if (void* sp = lz_scratch_resolved()) {
    uint32_t sbits = 0;
    HIP_TRY(hipMemcpy(&sbits, sp, sizeof(sbits), hipMemcpyDeviceToHost));
    if (sbits) HIP_TRY(hipMemset(sp, 0, sizeof(uint32_t)));
    bits |= sbits;
  }
  return status_of_bits(bits);
}

const char* sg_last_error(void) { return g_last_error.c_str(); }

sg_status sg_get_run_info(void* stream, sg_run_info* out) {
  if (!out) return fail(SG_EINVAL, "null output");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(st));
  std::memset(out, 0, sizeof(*out));
  Workspace* w = ws_find(st);
  if (!w) return SG_OK;
  Params p;
  HIP_TRY(hipMemcpy(&p, w->P, sizeof(p), hipMemcpyDeviceToHost));
  out->chunks = w->last_chunks;
  out->candidates = (int64_t)p.stat_candidates;
  out->slow_blocks = (int64_t)p.stat_slow;
  out->margin = p.margin;
  float d;
  std::memcpy(&d, &p.max_drift_bits, sizeof(d));
  out->max_drift = d;
  out->prefix_bits_max = w->last_kmax;
  out->free_bits_max = w->last_nmax;
  out->enum_launches = w->last_launches;
  out->enum_states = w->last_states;
  double ms = 0.0;
  for (int i = 0; i < w->ev_used; ++i) {
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, w->ev[2 * i], w->ev[2 * i + 1]));
    ms += t;
  }
  out->enum_ms = ms;
  out->max_chunk_candidates = p.max_chunk_cand;
  out->repeated_passes = p.stat_redo;
  return SG_OK;
}

void sg_set_kernel_timing(int enable) { g_timing = enable != 0; }

double sg_probe_valu(int op, int waves_per_simd) {
  if (op < 0 || op > 27 || waves_per_simd < 1 || waves_per_simd > 8) return -1.0;
  return probe_valu(op, waves_per_simd);
}

sg_status sg_debug_set_fill(void* stream, long long lanes) {
  g_last_error.clear();
  if (lanes < 0) return fail(SG_EINVAL, "lanes must be >= 0");
  Workspace* w = nullptr;
  const sg_status v = ws_get((hipStream_t)stream, 1, 1, 1, 1, &w);
  if (v != SG_OK) return v;
  std::lock_guard<std::mutex> lk(g_mu);
  for (int k = 0; k < 2; ++k) {
    w->fill[k] = lanes > 0 ? (int64_t)lanes : w->fill_dev[k];
    w->launch[k] = lanes > 0 ? (int64_t)lanes : kSearchLaunchFills * w->fill_dev[k];
  }
  w->tri_all = lanes > 0;
  return SG_OK;
}

sg_status sg_debug_set_margin_scale(void* stream, double scale) {
  g_last_error.clear();
  if (!(scale > 0.0) || !(scale <= 1.0)) return fail(SG_EINVAL, "scale must be in (0, 1]");
  Workspace* w = nullptr;
  const sg_status v = ws_get((hipStream_t)stream, 1, 1, 1, 1, &w);
  if (v != SG_OK) return v;
  std::lock_guard<std::mutex> lk(g_mu);
  w->margin_scale = (float)scale;
  return SG_OK;
}

sg_status sg_debug_set_batch_shift(int B, int N_max, int S, int shift) {
  g_last_error.clear();
  if (B < 1 || S < 1 || shift > 40) return fail(SG_EINVAL, "need B >= 1, S >= 1, shift <= 40");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  const auto key = std::make_tuple(dev, B, N_max, S);
  if (shift < 0) g_shift.erase(key);
  else g_shift[key] = shift;
  return SG_OK;
}

int sg_debug_plan(int N, int S, uint64_t lo, uint64_t hi, int64_t lanes_fill,
                  uint64_t* first_mask, int32_t* free_bits, int64_t* lanes, int cap) {
  if (N < 1 || N > SG_MAX_N || S < 1 || lo >= hi || hi > ((uint64_t)1 << N) || (lo % 64) != 0 ||
      lanes_fill < 1)
    return -1;
  const std::vector<PlanChunk> plan =
      plan_chunks(N, S, lo, hi, lanes_fill, search_block(N), lanes_fill);
  for (int i = 0; i < (int)plan.size() && i < cap; ++i) {
    if (first_mask) first_mask[i] = plan[i].first_mask;
    if (free_bits) free_bits[i] = plan[i].n;
    if (lanes) lanes[i] = plan[i].lanes;
  }
  return (int)plan.size();
}

}  // extern "C"
