/*
 * sg.h -- C ABI of the MI355X (gfx950) exhaustive Ising low-spectrum engine.
 *
 * The operation (arXiv:1904.03621, Sec. 2 Eq. (1) and Sec. 3 Algorithm 1):
 * for an Ising instance on an arbitrary graph with N spins,
 *
 *     E(s) = - sum_{i<j} J_ij s_i s_j - sum_i h_i s_i ,   s_i = +-1,
 *
 * enumerate all 2^N configurations and return the S lowest (S << 2^N)
 * together with their energies.
 *
 * Conventions shared by every entry point:
 *   - State masks: spin i (0-based) is bit i of a uint64 mask; a set bit
 *     means s_i = +1 (the thread-index encoding of Eqs. (4)-(6), least
 *     significant bit first).
 *   - J is a dense row-major N x N array; only the strict upper triangle
 *     J[i*N + j], i < j, is read (each unordered pair once, Eq. (1)); the
 *     diagonal and the lower triangle are ignored.  h has N entries.
 *   - Results are sorted ascending by the key (energy, mask): ties in energy
 *     are ordered by the mask, which makes the answer unique.
 *   - All array pointers are DEVICE pointers owned by the caller; the library
 *     never frees them.  `stream` is a hipStream_t passed as void* (NULL is
 *     the default stream).  Calls enqueue work on `stream` and return
 *     without waiting for it.
 *   - The return value is the synchronous validation status.  Errors found
 *     on the device (non-finite input, integer overflow risk, candidate
 *     buffer overflow, fp32 drift beyond its bound) are sticky per stream and
 *     are read back with sg_get_error, which waits for the stream.
 *   - The library owns a per-(device, stream) workspace that it allocates on
 *     first use and grows when a call needs more; it is released at process
 *     exit.  Calls on one stream are ordered; calls on different streams use
 *     different workspaces and may run concurrently.  Two host threads must
 *     not issue calls on the same stream at the same time.
 *   - Graph capture: a call enqueued while its stream captures a HIP graph
 *     allocates nothing; if the workspace is too small for it the call
 *     returns SG_EINVAL (size it first with sg_reserve or one eager call of
 *     the same shape).  From the first sg_reserve or captured call on, the
 *     workspace never frees a buffer: a later, larger eager call allocates
 *     new ones and keeps the old ones (which captured graphs still use)
 *     until the process ends.
 *   - SG_ECAPACITY: a chunk whose candidates overflow the buffer is walked
 *     again (up to two more times) with the threshold its partial merge
 *     tightened; the error is reported only if the last pass still
 *     overflows (extreme near-degeneracy).
 */
#ifndef SG_H
#define SG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SG_OK = 0,
    SG_EINVAL = 1,        /* bad argument (sizes, null pointers, ranges)      */
    SG_ENONFINITE = 2,    /* NaN or Inf in J or h (device-detected)           */
    SG_EOVERFLOW = 3,     /* integer instance: sum|J| + sum|h| >= 2^28        */
    SG_ENOMEM = 4,        /* workspace allocation failed                      */
    SG_EHIP = 5,          /* a HIP runtime call failed                        */
    SG_EUNSUPPORTED = 6,  /* no gfx950 device / unsupported configuration     */
    SG_EDRIFT = 7,        /* fp32 incremental drift exceeded its bound        */
    SG_ECAPACITY = 8      /* candidate buffer overflowed; result incomplete   */
} sg_status;

/* Largest number of spins accepted (Sec. 3: a state is the 64-bit code of its
 * spins; one bit short of that keeps every mask a non-negative signed 64-bit
 * integer, while range ends, unsigned, reach 2^63). */
#define SG_MAX_N 63
/* Largest S accepted by the single-instance search. */
#define SG_MAX_S (1 << 20)
/* Largest S accepted by the batched search. */
#define SG_MAX_S_BATCHED 4096

/*
 * sg_low_spectrum_f32 -- the S lowest states of a float32 instance
 * (Sec. 3, Algorithm 1; energy of Eq. (1)).
 *
 *   N            number of spins, 1 <= N <= SG_MAX_N
 *   J            device float[N*N], row-major, strict upper triangle read
 *   h            device float[N]
 *   S            number of states wanted, 1 <= S <= min(2^N, SG_MAX_S)
 *   states_out   device uint64[S]  masks, ascending by (energy, mask)
 *   energies_out device float[S]   energies of those states
 *
 * The enumeration accumulates energies incrementally in fp32 (block-start
 * values, with the states of a block in fixed point relative to the pruning
 * bound where a lane walks at least 10 spins: 16-bit fields, or 11/11/10-bit
 * fields from 20 spins on), re-anchors from scratch every 2^10 Gray-code
 * flips (2^14 in the fixed-point walks, whose fp32 part rounds far less
 * often), prunes with a margin that bounds the
 * accumulated rounding, and rescores every surviving candidate from scratch
 * in fp64; the returned energies are those fp64 values rounded to fp32 (-0
 * is returned as +0).
 */
sg_status sg_low_spectrum_f32(int N, const float *J, const float *h, int S,
                              uint64_t *states_out, float *energies_out,
                              void *stream);

/*
 * sg_low_spectrum_i32 -- the same search for an integer instance, computed
 * exactly in int32 (bit-exact energies and order).  Requires
 * sum_{i<j}|J_ij| + sum_i|h_i| < 2^28 (else SG_EOVERFLOW via sg_get_error).
 */
sg_status sg_low_spectrum_i32(int N, const int32_t *J, const int32_t *h, int S,
                              uint64_t *states_out, int32_t *energies_out,
                              void *stream);

/*
 * Range variants: the S lowest states among masks in [mask_lo, mask_hi)
 * only -- the chunk offset of Eq. (6).  A contiguous mask range is the unit
 * a multi-device run would hand to each device; the tests use it to check
 * slices of a 2^48 space against the oracle.  mask_lo and mask_hi must be
 * multiples of 64 (or mask_hi == 2^N), mask_lo < mask_hi <= 2^N, and
 * S <= mask_hi - mask_lo.
 */
sg_status sg_low_spectrum_range_f32(int N, const float *J, const float *h, int S,
                                    uint64_t mask_lo, uint64_t mask_hi,
                                    uint64_t *states_out, float *energies_out,
                                    void *stream);
sg_status sg_low_spectrum_range_i32(int N, const int32_t *J, const int32_t *h, int S,
                                    uint64_t mask_lo, uint64_t mask_hi,
                                    uint64_t *states_out, int32_t *energies_out,
                                    void *stream);

/*
 * Batched search: the S lowest states of each of B independent instances of
 * uneven size, in one sequence of launches on `stream` (about 2 log2(2^N_max)
 * kernels for the whole batch, whatever B is).  Every instance runs the same
 * search as sg_low_spectrum_f32 / _i32 and gets the same result.
 *
 *   B            number of instances, >= 1
 *   N_dev        device int32[B]: spins of instance b, 7 <= N_b <= N_max
 *   N_max        largest N_b (row stride of J), 7 <= N_max <= 40
 *   J            device float[B][N_max][N_max] (int32 for _i32); instance b
 *                uses its leading N_b x N_b block, strict upper triangle
 *   h            device float[B][N_max]; instance b uses its first N_b
 *   S            states per instance, 1 <= S <= SG_MAX_S_BATCHED, S <= 2^N_b
 *   states_out   device uint64[B][S], energies_out device float[B][S]
 *
 * The instance sizes are read on the device only, so the enqueued work
 * depends on (B, N_max, S) alone: one capture into a HIP graph serves every
 * batch of that shape.  Bad N_b or S > 2^N_b are reported as SG_EINVAL by
 * sg_get_error.  The workspace must already be large enough before a graph
 * capture (run one call of the same shape first).
 */
sg_status sg_low_spectrum_batched_f32(int B, const int32_t *N_dev, int N_max, const float *J,
                                      const float *h, int S, uint64_t *states_out,
                                      float *energies_out, void *stream);
sg_status sg_low_spectrum_batched_i32(int B, const int32_t *N_dev, int N_max, const int32_t *J,
                                      const int32_t *h, int S, uint64_t *states_out,
                                      int32_t *energies_out, void *stream);

/*
 * Exact log partition function of B instances of N spins (fp32 couplings):
 *   Z_b(beta) = sum over all 2^N states s of exp(-beta E_b(s)),
 * the normaliser of the Boltzmann distribution at inverse temperature beta
 * (Sec. 5.2, Eq. 10) for the energy of Eq. (1).  The S lowest states are found
 * first (the batched search); log Z is then computed as
 *   log Z = -beta E0 + log sum_s exp(-beta (E(s) - E0)),
 * with E0 the lowest energy, so that no weight exceeds 1.
 *
 *   B            number of instances, >= 1
 *   N            spins of every instance, 7 <= N <= 40
 *   J            device float[B][N][N], strict upper triangle read
 *   h            device float[B][N]
 *   n_beta       number of inverse temperatures, 1 <= n_beta <= 4
 *   beta         device float[n_beta], each finite and > 0 (else SG_EINVAL
 *                via sg_get_error)
 *   S            lowest states returned per instance, 1 <= S <=
 *                SG_MAX_S_BATCHED, S <= 2^N
 *   logz_out     device double[B][n_beta]
 *   e0_out       device float[B]: the lowest energy E0 (= energies_out[b][0])
 *   states_out   device uint64[B][S], energies_out device float[B][S]: the
 *                result of sg_low_spectrum_batched_f32 on the same batch
 *
 * The walk keeps its energy chain in fp64 and evaluates each weight in fp32
 * (shifted energy rounded to fp32, hardware exp2); block sums of 1024 weights
 * (256 when N = 8, 9 or n_beta = 4; 64 when N = 7) are fp32, every longer sum
 * is fp64.  Relative error of
 * log Z: about 1e-7.  All
 * buffers are caller-owned; work is enqueued on `stream`.
 */
sg_status sg_logz_forward_f32(int B, int N, const float *J, const float *h, int n_beta,
                              const float *beta, int S, double *logz_out, float *e0_out,
                              uint64_t *states_out, float *energies_out, void *stream);

/*
 * Gradient of L = sum_{b,k} g[b][k] log Z_b(beta_k) with respect to J and h:
 *   dL/dJ_ij = sum_k g[b][k] beta_k <s_i s_j>_k   (i < j)
 *   dL/dh_i  = sum_k g[b][k] beta_k <s_i>_k
 * with <.>_k the average under the Boltzmann distribution at beta_k (Sec. 5.2,
 * Eq. 10).  The enumeration is walked again (no per-state storage) with the
 * combined weight sum_k (g[b][k] beta_k / Z_k) exp(-beta_k E(s)).
 *
 *   B, N, J, h, n_beta, beta  as for sg_logz_forward_f32
 *   e0           device float[B]: e0_out of the forward call
 *   logz         device double[B][n_beta]: logz_out of the forward call
 *   grad_logz    device double[B][n_beta]: g, the incoming gradient
 *   grad_J       device float[B][N][N]: written for i < j, zeros elsewhere
 *   grad_h       device float[B][N]
 *
 * Moments are summed in fp32 inside a 64-state block (and over the four
 * blocks of a 256-state record) and in fp64 beyond.
 * All buffers are caller-owned; work is enqueued on `stream`.
 */
sg_status sg_logz_backward_f32(int B, int N, const float *J, const float *h, int n_beta,
                               const float *beta, const float *e0, const double *logz,
                               const double *grad_logz, float *grad_J, float *grad_h,
                               void *stream);

/*
 * The same gradients as sg_logz_backward_f32, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight training or
 * serving loops, harnesses that forbid hipMalloc.  The call allocates
 * nothing: its block records, bq tables, weights, fp64 accumulators and
 * error word live in a static device array of SG_LOGZ_SCRATCH_BYTES bytes
 * that each device running the library holds until the process ends (its
 * device address is looked up once per device, on the first call there).
 * Arguments, outputs and results are those of sg_logz_backward_f32 on the
 * same stream (same decomposition, same kernels).
 *
 *   SG_EINVAL  also when B and N need more than SG_LOGZ_SCRATCH_BYTES: at
 *              most B (14 KiB + 8 (N^2 + N) bytes), so every B <= 1200 fits
 *              for N <= 40 (the message gives the bytes a refused call needs).
 *
 * All calls on one device share that device's array and it keeps the last
 * call's contents (the accumulators are cleared by every call): calls that
 * overlap on one device -- on different streams, or from different host
 * threads -- race and must be serialised by the caller.  Device-side errors
 * are ORed into the array's error word, which sg_get_error reports and
 * clears (pass it the stream of the call, so that it waits for it).
 */
#define SG_LOGZ_SCRATCH_BYTES (32ull << 20)

sg_status sg_logz_backward_noalloc_f32(int B, int N, const float *J, const float *h, int n_beta,
                                       const float *beta, const float *e0, const double *logz,
                                       const double *grad_logz, float *grad_J, float *grad_h,
                                       void *stream);

/*
 * QUBO front end (Sec. 2, Eqs. 2-3): the S lowest of
 *     F(q) = - sum_{i<j} a_ij q_i q_j - sum_i b_i q_i ,   q_i in {0, 1},
 * over all 2^N binary vectors, found by the Ising search on the instance of
 * Eq. (3) (J = a/4, h_i = b_i/2 + sum_{j!=i} a_ij/4, formed on the device in
 * fp64 and rounded to fp32) and rescored in the QUBO form.
 *
 *   N            1 <= N <= SG_MAX_N
 *   A            device float[N][N], strict upper triangle a_ij (i < j) read
 *   b            device float[N]
 *   S            1 <= S <= SG_MAX_S_BATCHED, S <= 2^N
 *   states_out   device uint64[S]: bit i = q_i
 *   energies_out device float[S]: F in fp64 rounded to fp32, ascending by
 *                (F, mask)
 *
 * When h has to be rounded to fp32 the set may differ from the exact QUBO
 * answer only among states within N ulp of the S-th value; integer a and b
 * (and any dyadic ones of moderate range) are exact.  Errors as for
 * sg_low_spectrum_f32.
 */
sg_status sg_low_spectrum_qubo_f32(int N, const float *A, const float *b, int S,
                                   uint64_t *states_out, float *energies_out, void *stream);

/* Largest number of energy bins of sg_density_of_states_i32. */
#define SG_MAX_DOS_BINS 8192

/*
 * Exact density of states of an integer instance: the number of the 2^N
 * configurations at each energy of Eq. (1), all enumerated (the quantity the
 * entropic population annealing comparison of Sec. 5.2 estimates).
 *
 *   N            1 <= N <= SG_MAX_N; int32 J (N x N, strict upper triangle
 *                read) and h as for sg_low_spectrum_i32, with
 *                sum|J| + sum|h| < 2^28 (else SG_EOVERFLOW via sg_get_error)
 *   e_min        energy of bin 0
 *   n_bins       1 <= n_bins <= SG_MAX_DOS_BINS
 *   counts_out   device uint64[n_bins]: counts_out[k] = number of
 *                configurations with E = e_min + k (overwritten)
 *
 * The bins must cover [-B, B] with B = sum_{i<j}|J_ij| + sum_i|h_i| (which no
 * |E| exceeds; sg_energy_bound_i32 computes it), else SG_EINVAL via
 * sg_get_error and the counts stay zero.  Work is enqueued on `stream`.
 */
sg_status sg_density_of_states_i32(int N, const int32_t *J, const int32_t *h, long long e_min,
                                   int n_bins, unsigned long long *counts_out, void *stream);

/*
 * B = sum_{i<j} |J_ij| + sum_i |h_i| of an int32 instance, written to the
 * device int64 `bound_out` (enqueued on `stream`).
 */
sg_status sg_energy_bound_i32(int N, const int32_t *J, const int32_t *h, long long *bound_out,
                              void *stream);

/*
 * Sizes the library's workspace of (current device, stream) for every later
 * call on that stream with B <= B_max, N <= N_max and S <= S_max (single,
 * batched and log Z calls).  Calls within those limits then allocate nothing,
 * so they can be captured into a HIP graph.  Synchronous; returns SG_EINVAL
 * for out-of-range limits and SG_ENOMEM / SG_EHIP if allocation fails.  The
 * workspace is owned by the library and lives until the process ends; once
 * reserved it keeps every buffer a captured graph may use (see "Graph
 * capture" above).
 */
sg_status sg_reserve(int B_max, int N_max, int S_max, void *stream);

/*
 * Tuner of the batched search: times sg_low_spectrum_batched_f32 on this
 * batch for the level geometries around the default (free spins per lane n =
 * log2(level size) - shift; by default shift = max(12, ceil(log2(4 L / B))),
 * L the device's resident lanes; the tuner tries that shift -3 .. +3) and keeps the
 * fastest for later batched calls on this device with the same B, N_max and
 * S; *shift_out is the choice.  Results do not depend on the geometry (the
 * search is exact).  Synchronous; allocates scratch and runs the search 21
 * times; call it before capturing a graph of batched calls (the geometry fixes
 * the launch sequence).  Arguments as for sg_low_spectrum_batched_f32.
 */
sg_status sg_tune_batched_f32(int B, const int32_t *N_dev, int N_max, const float *J,
                              const float *h, int S, int *shift_out, void *stream);

/* Waits for `stream`, then returns and clears the sticky device error of the
 * calls enqueued on it, together with that of the current device's static
 * scratch (sg_logz_backward_noalloc_f32) (SG_OK if none). */
sg_status sg_get_error(void *stream);

/* Human-readable text of the last failure on the calling thread ("" if none). */
const char *sg_last_error(void);

/* Counters of the last search enqueued on `stream` (waits for the stream). */
typedef struct {
    int64_t chunks;          /* enumeration launches                          */
    int64_t candidates;      /* states that passed the in-kernel test         */
    int64_t slow_blocks;     /* wave-blocks that took the exact re-walk path  */
    double  margin;          /* fp32 pruning margin used (0 for int32)        */
    double  max_drift;       /* largest |incremental - fresh| at re-anchors   */
    int32_t prefix_bits_max; /* largest k = N - n used                        */
    int32_t free_bits_max;   /* largest n used                                */
    int64_t enum_launches;   /* enumeration kernel launches                   */
    double  enum_states;     /* states covered by those launches              */
    double  enum_ms;         /* their summed duration (HIP events; 0 unless
                                kernel timing is on)                          */
    int64_t max_chunk_candidates; /* most candidates one chunk produced       */
    int64_t repeated_passes; /* chunks walked again because their candidates
                                overflowed the buffer (instance 0)            */
} sg_run_info;
sg_status sg_get_run_info(void *stream, sg_run_info *out);

/* Kernel timing switch (process-wide, default off): when on, each
 * enumeration launch is bracketed by HIP events on its stream and
 * sg_get_run_info reports their summed duration. */
void sg_set_kernel_timing(int enable);

/*
 * Measurement hook: issue rate of one VALU instruction kind on the current
 * device, in lane-instructions per second (0 v_add_f32, 1 v_min3_f32,
 * 2 v_add_u32, 3 v_min3_i32, 4 v_fma_f32, 5 v_min_f32, 6 v_or_b32,
 * 7 v_or3_b32, 8 v_add3_u32, 9 v_max3_f32, 10 v_min_i32, 11 v_sub_f32,
 * 12 v_and_or_b32, 13 v_med3_f32, 14 v_pk_add_u16, 15 v_pk_min_i16,
 * 16 v_exp_f32, 17 v_sub_u32, 18 v_and_b32, 19 v_cvt_i32_f32,
 * 20 v_lshl_add_u32), or of an instruction mix of the walk's steps, 8
 * independent chains per lane (21: two v_add_f32 and one v_min3_f32 per two
 * states, the fp32 walk; 22: v_add_u32, v_and_b32, v_sub_u32, v_and_b32 per two
 * steps, the walk over two 16-bit fields per word; 23 and 24: 22 with one
 * and two chains per lane; 25: 21 with one chain per lane; 26: 23 with 57
 * more registers live; 27: 23 as one straight run of 1024 steps), with
 * `waves_per_simd` (1..8) resident waves on every SIMD.
 * Synchronous (own stream); returns < 0 on error.  Context for the
 * enumeration kernel's roofline: which instructions issue at the doubled
 * rate.
 */
double sg_probe_valu(int op, int waves_per_simd);

/*
 * Test hooks (not compute calls).  They change how later calls lay out their
 * work, never what a correct call computes, so that instances small enough
 * for the CPU oracle can run the code paths of the large workloads.
 *
 * sg_debug_set_fill: the number of lanes the work plans of (current device,
 * stream) assume (lanes >= 1; 0 restores the device's own values): the
 * resident lanes of the density of states and log Z, and the lanes a single
 * search plans its chunks for (by default 8 times the resident lanes).  While it is set, every chunk of 14 or more free spins takes the
 * three-field walk (by default only chunks of 20 or more that launch at
 * least the resident lanes).  The single search, the density of
 * states and log Z give each lane more free spins when there are fewer lanes
 * to fill: with lanes = 4 a search of N = 24 walks up to 2^21 states per
 * lane (block boundaries, high-spin fields, fp32 re-anchors), and a log Z
 * batch of one N = 20 instance runs 14 free spins per lane at lanes = 64.
 *
 * sg_debug_set_margin_scale: multiplies the fp32 pruning margin of later
 * searches on (current device, stream) by scale, 0 < scale <= 1 (1
 * restores).  Below 1 the margin may no longer bound the walk's rounding:
 * results may then be wrong, and the drift guard reports SG_EDRIFT through
 * sg_get_error once a measured drift exceeds the scaled margin.  Every kernel
 * still runs to its end.
 *
 * sg_debug_set_batch_shift: the level shift of batched calls with this (B,
 * N_max, S) on the current device, as sg_tune_batched_f32 would set it
 * (0 <= shift <= 40; shift < 0 restores the default).  A small shift gives
 * the lanes of a small batch up to 16 free spins.
 */
sg_status sg_debug_set_fill(void *stream, long long lanes);
sg_status sg_debug_set_margin_scale(void *stream, double scale);
sg_status sg_debug_set_batch_shift(int B, int N_max, int S, int shift);

/*
 * Test hook (not a compute call): the chunk plan the library would use for a
 * search of [mask_lo, mask_hi) with S states on a device with `lanes_fill`
 * resident lanes.  Writes up to `cap` triples (first_mask, free_bits n,
 * lanes L), chunk c covering [first_mask, first_mask + L * 2^n); returns the
 * number of chunks (which may exceed cap), or -1 on bad arguments.
 */
int sg_debug_plan(int N, int S, uint64_t mask_lo, uint64_t mask_hi, int64_t lanes_fill,
                  uint64_t *first_mask, int32_t *free_bits, int64_t *lanes, int cap);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
