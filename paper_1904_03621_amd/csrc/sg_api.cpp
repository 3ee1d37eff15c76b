// sg_api.cpp -- host side of the C ABI (include/sg.h): argument validation,
// per-(device, stream) workspace, the chunk plan and the kernel sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/sg.h"
#include "sg_internal.h"

namespace sg {
hipError_t launch_prep(bool isint, const void* J, const void* h, int N, int S, Params* P,
                       uint32_t* qtab, hipStream_t st);
hipError_t launch_tables(bool isint, const void* J, const void* h, int N, int nmax,
                         uint32_t* table, hipStream_t st);
hipError_t launch_enum(bool isint, const void* J, const void* h, int N, const Chunk& ch,
                       const uint32_t* table, const uint32_t* qtab, Params* P, uint64_t* cand,
                       uint32_t cap, hipStream_t st);
hipError_t launch_direct(int N, uint64_t lo, uint64_t hi, Params* P, uint64_t* cand, uint32_t cap,
                         hipStream_t st);
hipError_t launch_score(bool isint, const void* J, const void* h, int N, Params* P,
                        const uint64_t* cand, uint32_t cap, uint32_t* skey, uint64_t* smask,
                        int grid, hipStream_t st);
hipError_t launch_merge(Params* P, int S, uint32_t cap, uint32_t* skey, uint64_t* smask,
                        uint32_t* rkey, uint64_t* rmask, uint32_t* tkey, uint64_t* tmask,
                        hipStream_t st);
hipError_t launch_finalize(bool isint, const Params* P, int S, const uint32_t* rkey,
                           const uint64_t* rmask, uint64_t* states_out, void* energies_out,
                           uint32_t* sticky, hipStream_t st);
int enum_occupancy(bool isint);
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

struct PlanChunk {
  uint64_t first_mask;
  int n;
  int64_t lanes;
};

// Chunks of [lo, hi) in ascending mask order.  The first chunk has at least
// max(S, 4096) states (it runs with no threshold, so every state is a
// candidate); each next chunk is as large as everything processed before it,
// so that the expected number of candidates per chunk stays near S, until
// the chunk reaches `fill` lanes of 2^nmax states; from then on chunks have
// fill lanes each.  Every chunk is [first, first + L 2^n) with first a
// multiple of 2^n, and lanes cover consecutive prefixes.
std::vector<PlanChunk> plan_chunks(int N, int S, uint64_t lo, uint64_t hi, int64_t fill) {
  std::vector<PlanChunk> out;
  const int nmax = std::min(kMaxFree, N);
  if (fill < kWaveLanes) fill = kWaveLanes;
  const int fill_log = ilog2_floor((uint64_t)fill);
  uint64_t target = 4096;
  while (target < (uint64_t)S) target <<= 1;
  const uint64_t big = (uint64_t)fill << nmax;
  uint64_t cur = lo;
  while (cur < hi) {
    const uint64_t rem = hi - cur;
    PlanChunk c{};
    c.first_mask = cur;
    const uint64_t unit = (uint64_t)1 << nmax;
    if (target >= big && (cur & (unit - 1)) == 0 && rem >= unit) {
      // near the end shrink n rather than the lane count, so that the last
      // chunks still fill the device
      int n = nmax;
      while (n > kU && (rem >> n) < (uint64_t)fill) --n;
      c.n = n;
      c.lanes = (int64_t)std::min<uint64_t>((uint64_t)fill, rem >> n);
    } else {
      uint64_t size = std::min<uint64_t>(target, big);
      if (cur != 0) size = std::min<uint64_t>(size, cur & (~cur + 1));
      while (size > rem) size >>= 1;
      const int slog = ilog2_floor(size);
      int n = slog - fill_log;
      n = std::max(n, kU);
      n = std::min(n, nmax);
      n = std::min(n, slog);
      c.n = n;
      c.lanes = (int64_t)(size >> n);
    }
    out.push_back(c);
    cur += (uint64_t)c.lanes << c.n;
    target = std::max<uint64_t>(target, 2 * (cur - lo));
  }
  return out;
}

// --------------------------------------------------------------- workspace

struct Workspace {
  int device = -1;
  Params* P = nullptr;
  uint32_t* sticky = nullptr;
  uint32_t* qtab = nullptr;
  uint32_t* table = nullptr;
  uint64_t* cand = nullptr;
  uint32_t* skey = nullptr;
  uint64_t* smask = nullptr;
  uint32_t cap = 0;
  uint32_t* rkey = nullptr;
  uint64_t* rmask = nullptr;
  uint32_t* tkey = nullptr;
  uint64_t* tmask = nullptr;
  int rec_cap = 0;
  int64_t fill[2] = {0, 0};
  int cus = 0;
  // last run
  int64_t last_chunks = 0;
  int last_kmax = 0, last_nmax = 0;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

constexpr uint32_t kCandCapMin = 1u << 22;

sg_status ws_create(int dev, Workspace* w) {
  w->device = dev;
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SG_EUNSUPPORTED,
                std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  w->cus = prop.multiProcessorCount;
  for (int k = 0; k < 2; ++k) {
    const int occ = enum_occupancy(k == 1);
    w->fill[k] = (int64_t)w->cus * std::max(occ, 1) * kEnumBlock;
  }
  HIP_TRY(hipMalloc(&w->P, sizeof(Params)));
  HIP_TRY(hipMalloc(&w->sticky, sizeof(uint32_t)));
  HIP_TRY(hipMemset(w->sticky, 0, sizeof(uint32_t)));
  HIP_TRY(hipMalloc(&w->qtab, 2 * kBlockSteps * sizeof(uint32_t)));
  const size_t recs = ((size_t)1 << (kMaxFree - kU + 1)) - 1;
  HIP_TRY(hipMalloc(&w->table, recs * kRecWords * sizeof(uint32_t)));
  return SG_OK;
}

// The workspace of (current device, stream), created on first use and grown
// to hold S record entries and the candidate buffer.  Growing frees the old
// buffers (hipFree waits for the device), so it never races earlier calls.
sg_status ws_get(hipStream_t st, int S, Workspace** out) {
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
      if (w->P) (void)hipFree(w->P);
      if (w->sticky) (void)hipFree(w->sticky);
      if (w->qtab) (void)hipFree(w->qtab);
      if (w->table) (void)hipFree(w->table);
      delete w;
      return s;
    }
    g_ws[key] = w;
  }
  // candidate capacity: the first chunk (all candidates) has < 2 max(S, 4096)
  uint32_t need = kCandCapMin;
  while (need < 8u * (uint32_t)S) need <<= 1;
  if (w->cap < need) {
    if (w->cand) {
      HIP_TRY(hipFree(w->cand));
      HIP_TRY(hipFree(w->skey));
      HIP_TRY(hipFree(w->smask));
    }
    HIP_TRY(hipMalloc(&w->cand, (size_t)need * sizeof(uint64_t)));
    HIP_TRY(hipMalloc(&w->skey, (size_t)need * sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&w->smask, (size_t)need * sizeof(uint64_t)));
    w->cap = need;
  }
  if (w->rec_cap < S) {
    if (w->rkey) {
      HIP_TRY(hipFree(w->rkey));
      HIP_TRY(hipFree(w->rmask));
      HIP_TRY(hipFree(w->tkey));
      HIP_TRY(hipFree(w->tmask));
    }
    HIP_TRY(hipMalloc(&w->rkey, (size_t)S * sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&w->rmask, (size_t)S * sizeof(uint64_t)));
    HIP_TRY(hipMalloc(&w->tkey, (size_t)S * sizeof(uint32_t)));
    HIP_TRY(hipMalloc(&w->tmask, (size_t)S * sizeof(uint64_t)));
    w->rec_cap = S;
  }
  *out = w;
  return SG_OK;
}

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

sg_status run_search(bool isint, int N, const void* J, const void* h, int S, uint64_t lo,
                     uint64_t hi, uint64_t* states_out, void* energies_out, void* stream) {
  g_last_error.clear();
  sg_status v = validate(N, J, h, S, lo, hi, states_out, energies_out);
  if (v != SG_OK) return v;
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = nullptr;
  v = ws_get(st, S, &w);
  if (v != SG_OK) return v;

  HIP_TRY(launch_prep(isint, J, h, N, S, w->P, w->qtab, st));
  const int score_grid = std::max(1, w->cus) * 4;
  int64_t nchunks = 0;
  int kmax = 0, nmaxu = 0;
  if (N < kU) {
    HIP_TRY(launch_direct(N, lo, hi, w->P, w->cand, w->cap, st));
    HIP_TRY(launch_score(isint, J, h, N, w->P, w->cand, w->cap, w->skey, w->smask, score_grid, st));
    HIP_TRY(launch_merge(w->P, S, w->cap, w->skey, w->smask, w->rkey, w->rmask, w->tkey, w->tmask,
                         st));
    nchunks = 1;
  } else {
    const int nmax = std::min(kMaxFree, N);
    HIP_TRY(launch_tables(isint, J, h, N, nmax, w->table, st));
    const std::vector<PlanChunk> plan = plan_chunks(N, S, lo, hi, w->fill[isint ? 1 : 0]);
    for (const PlanChunk& pc : plan) {
      Chunk ch{};
      ch.first_mask = pc.first_mask;
      ch.prefix_base = pc.first_mask >> pc.n;
      ch.lanes = pc.lanes;
      ch.n = pc.n;
      ch.table_offset = (1 << (pc.n - kU)) - 1;
      HIP_TRY(launch_enum(isint, J, h, N, ch, w->table, w->qtab, w->P, w->cand, w->cap, st));
      HIP_TRY(launch_score(isint, J, h, N, w->P, w->cand, w->cap, w->skey, w->smask, score_grid,
                           st));
      HIP_TRY(launch_merge(w->P, S, w->cap, w->skey, w->smask, w->rkey, w->rmask, w->tkey,
                           w->tmask, st));
      kmax = std::max(kmax, N - pc.n);
      nmaxu = std::max(nmaxu, pc.n);
    }
    nchunks = (int64_t)plan.size();
  }
  HIP_TRY(launch_finalize(isint, w->P, S, w->rkey, w->rmask, states_out, energies_out, w->sticky,
                          st));
  w->last_chunks = nchunks;
  w->last_kmax = kmax;
  w->last_nmax = nmaxu;
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

sg_status sg_get_error(void* stream) {
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(st));
  Workspace* w = ws_find(st);
  if (!w) return SG_OK;
  uint32_t bits = 0;
  HIP_TRY(hipMemcpy(&bits, w->sticky, sizeof(bits), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(w->sticky, 0, sizeof(uint32_t)));
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
  return SG_OK;
}

int sg_debug_plan(int N, int S, uint64_t lo, uint64_t hi, int64_t lanes_fill,
                  uint64_t* first_mask, int32_t* free_bits, int64_t* lanes, int cap) {
  if (N < kU || N > SG_MAX_N || S < 1 || lo >= hi || hi > ((uint64_t)1 << N) || (lo % 64) != 0 ||
      lanes_fill < 1)
    return -1;
  const std::vector<PlanChunk> plan = plan_chunks(N, S, lo, hi, lanes_fill);
  for (int i = 0; i < (int)plan.size() && i < cap; ++i) {
    if (first_mask) first_mask[i] = plan[i].first_mask;
    if (free_bits) free_bits[i] = plan[i].n;
    if (lanes) lanes[i] = plan[i].lanes;
  }
  return (int)plan.size();
}

}  // extern "C"
