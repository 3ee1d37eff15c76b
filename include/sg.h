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
 *     different workspaces and may run concurrently.
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

/* Largest number of spins accepted (Sec. 1 / abstract: N <= 50 in practice;
 * masks are 64-bit). */
#define SG_MAX_N 56
/* Largest S accepted by the single-instance search. */
#define SG_MAX_S (1 << 20)

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
 * The enumeration accumulates energies incrementally in fp32 with a
 * from-scratch re-anchor every 2^16 Gray-code flips, prunes with a margin
 * that bounds the accumulated rounding, and rescores every surviving
 * candidate from scratch in fp64; the returned energies are those fp64
 * values rounded to fp32 (-0 is returned as +0).
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

/* Waits for `stream`, then returns and clears the sticky device error of the
 * calls enqueued on it (SG_OK if none). */
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
} sg_run_info;
sg_status sg_get_run_info(void *stream, sg_run_info *out);

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
