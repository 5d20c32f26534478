/*
 * qft.h - C ABI of the MI355X (gfx950) improved-QFT DFT library.
 *
 * The library computes, for complex signals x of length N = 2^r (r >= 1),
 *
 *     X(k) = sum_{n=0}^{N-1} x(n) exp(-2*pi*i*n*k/N),   k = 0..N-1
 *
 * unnormalised, in natural order (Pasquini, "Improved QFT algorithm for
 * power-of-two FFT", Sec. 2.1, eq. qft_0A with theta = 2*pi/N, eq. qft_0D),
 * by the improved Quick Fourier Transform of Sec. 5: the real/imaginary split
 * and real fold of Sec. 4.1-4.2, the DCT-0/DST-0 recursion with the extra
 * even/odd time-index decomposition of Sec. 5.2, and the secant conversion
 * (eq. qft_38A) applied only to odd-time/odd-harmonic signals.  All
 * arithmetic on the GPU is FP32; the N/4 trigonometric constants of Sec. 6.1
 * are generated on the host in FP64 and rounded once to FP32.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Data layout: transform-major and contiguous.  For a uniform plan element
 *    (b, n) lives at element offset b*N + n.  For an uneven plan transform i
 *    starts at the exclusive prefix sum of 2^log2n[j], j < i.
 *  - Element types: QFT_C32 = interleaved {float re, im} (8 bytes);
 *    QFT_C16 = interleaved {_Float16 re, im} (4 bytes, IEEE binary16),
 *    converted to FP32 on load and rounded to nearest-even on store.
 *  - Pointers passed to exec are DEVICE pointers on the plan's device.  The
 *    caller owns them.  `in` is only written when in == out (in-place);
 *    any other overlap of the two ranges is rejected.
 *  - `stream` is a hipStream_t (NULL = the null stream).  exec is
 *    asynchronous and stream-ordered; it never synchronises and never
 *    allocates device memory, so it may be captured in a HIP graph.
 *  - One exec may be in flight per plan at a time (the plan owns scratch
 *    memory); different plans may run concurrently.
 *  - Errors are returned as status codes, never by abort.  Arguments are
 *    validated before any HIP call, so invalid calls have no side effects.
 */
#ifndef QFT_H
#define QFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qft_plan_s* qft_plan_t;

typedef enum {
    QFT_SUCCESS = 0,
    QFT_ERROR_INVALID_VALUE = 1, /* null pointer, batch/count <= 0, bad dtype (QFT_I32 is
                                    accepted by qft_plan_create only) */
    QFT_ERROR_INVALID_SIZE = 2,  /* log2n outside [1, QFT_MAX_LOG2N] */
    QFT_ERROR_ALIGNMENT = 3,     /* pointer not aligned to the element size */
    QFT_ERROR_OVERLAP = 4,       /* in/out partially overlap */
    QFT_ERROR_ALLOC = 5,         /* device or host allocation failed */
    QFT_ERROR_HIP = 6,           /* a HIP runtime call failed: qft_last_hip_error() */
    QFT_ERROR_UNSUPPORTED = 7,   /* device is not gfx950 / feature not built */
    QFT_ERROR_SCRATCH = 8        /* qft_exec_fwd_static: beyond its static scratch */
} qft_status;

typedef enum {
    QFT_C32 = 0, /* complex FP32 storage, FP32 compute */
    QFT_C16 = 1, /* complex FP16 storage, FP32 compute */
    QFT_I32 = 2  /* fixed point: complex int32 storage and integer arithmetic */
} qft_dtype;

#define QFT_MAX_LOG2N 24

/*
 * Plan for `batch` transforms of length N = 2^log2n each (Sec. 2.1 problem
 * statement).  Allocates the device constant table (Sec. 6.1: N/4 constants,
 * the secants 1/(2 cos(2*pi*q/N)) of eq. qft_38A and cos(2*pi/8)) and, for N
 * beyond one workgroup's local memory, a device scratch of batch*N complex
 * FP32 values (N = 2^15, 2^16) or 2*batch*N (N > 2^16).  `device` is a HIP
 * device ordinal.  On success *plan receives
 * a handle owned by the caller (free with qft_plan_destroy); on failure
 * *plan is set to NULL.
 */
qft_status qft_plan_create(qft_plan_t* plan, int log2n, int64_t batch, qft_dtype dtype,
                           int device);

/*
 * Fixed point (dtype QFT_I32; Sec. 1 and Sec. 7 recommend the method where a
 * multiplication costs more than an addition).  Uniform plans only, 1 <=
 * log2n <= 16 (else QFT_ERROR_INVALID_SIZE); elements are interleaved
 * {int32 re, im} (8 bytes).  Every addition and subtraction wraps modulo
 * 2^32; the only multiplications are the secant conversions (eq. qft_38A)
 * and the N = 8 base cases, by block-scaled constants: slice L (periodization
 * 8L, the constants 1/(2 cos(pi (2m+1)/(4L))), m < L) has one shift s_L = 30 -
 * e_L, e_L the binary exponent of its largest constant, and mantissas
 * H = floor(h 2^s_L + 1/2) (FP64, rounded once); a product is the 64-bit
 * w H rounded half up at bit s_L, kept to 32 bits.  The output is the exact
 * DFT of the integer input up to those roundings, and is bit-identical to
 * the integer recursion in the paper's order for any input.  Without
 * overflow, i.e. for |Re x|, |Im x| <= 2^(28 - log2n) (the largest growth of
 * an intermediate measured over all inputs is below 1.4 N per real signal
 * for N <= 2^11, growing about 17% per doubling), it approximates X within
 * the rounding of about N log2 N - 3N products.  The plan allocates the
 * integer table and, for log2n > 12, 2*batch*N int32 pairs of scratch; exec
 * runs the transforms in LDS up to 2^12 points (2^12 / N of them per
 * workgroup), beyond that one workgroup per transform.
 * qft_exec_bwd gives the adjoint by the same swap identity as below.
 */

/*
 * Plan for `count` transforms of possibly different lengths 2^log2n[i]
 * (host array, read during the call only), packed back to back in the given
 * order.  Every log2n[i] must lie in [1, QFT_MAX_LOG2N].  Transforms of up to
 * 2^14 points run in persistent tile-kernel launches over size-sorted work
 * lists (whole transforms in one workgroup's local memory); longer ones use
 * the two-pass (2^15, 2^16) or multi-pass path, one after the other.  The
 * plan holds several schedules (see qft_plan_schedules); schedule 0 runs
 * every transform of up to 2^14 points in ONE persistent launch.
 */
qft_status qft_plan_create_uneven(qft_plan_t* plan, const int32_t* log2n, int64_t count,
                                  qft_dtype dtype, int device);

/* X = F x: forward transform of every signal of the plan (eq. qft_0A). */
qft_status qft_exec_fwd(qft_plan_t plan, const void* in, void* out, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): X = F x for
 * `batch` transforms of N = 2^log2n points, with no plan and no allocation.
 * The same kernels as qft_exec_fwd on a uniform plan run on device pointers
 * `in`/`out` of the CURRENT device (layout, dtype, in == out and the error
 * codes as there).  Instead of a plan's memory they use a static scratch
 * array of 64 MiB per GPU (a device symbol of the library, held until the
 * process ends): the constant table, recomputed on `stream` by every call,
 * and for log2n = 15, 16 the two-pass heap buffer.  Limits: log2n <= 16, and
 * batch * 2^log2n <= 2^23 - 2^14 points for log2n = 15, 16; larger requests
 * return QFT_ERROR_SCRATCH.  Every call on one GPU uses that GPU's single
 * copy, so calls that overlap in time on one GPU (other streams, other host
 * threads) race on it; the scratch needs no clearing (every cell a call reads
 * is written by that call first).  The first call on each device looks up
 * the scratch's device address and the resident grid (runtime queries, no
 * stream work); make that call before capturing a graph.
 */
qft_status qft_exec_fwd_static(int log2n, int64_t batch, qft_dtype dtype, const void* in,
                               void* out, void* stream);

/*
 * x = F^H X: the adjoint (conjugate transpose), exp(+2*pi*i*n*k/N), also
 * unnormalised, so exec_bwd(exec_fwd(x)) = N x.  It runs the same improved-QFT
 * plan on swap(X) and swaps the result, swap(a + ib) = b + ia, since
 * F^H g = swap(F swap(g)).
 */
qft_status qft_exec_bwd(qft_plan_t plan, const void* in, void* out, void* stream);

/* Frees every device and host resource of the plan.  NULL is accepted. */
qft_status qft_plan_destroy(qft_plan_t plan);

/*
 * Plan figures (any output pointer may be NULL):
 *   total_points  sum of N over the plan's transforms;
 *   algo_bytes    bytes one exec must move at minimum (read + write of every
 *                 element once: 2 * total_points * element size);
 *   flops_5nlogn  sum of 5 N log2 N (the usual FFT flop convention);
 *   flops_actual  sum of 4 N log2 N - 6N + 8, the improved QFT's real
 *                 additions plus multiplications (Table 2, CDFT row).
 */
qft_status qft_plan_info(qft_plan_t plan, int64_t* total_points, int64_t* algo_bytes,
                         double* flops_5nlogn, double* flops_actual);

/*
 * Schedules.  A plan holds one or more schedules: ways to run the same
 * computation that differ only in how the work is cut into launches and
 * passes (every schedule of a plan gives bit-identical results).
 *  - Uniform plans, N <= 2^14: schedule 0 ("t<T>:<r>") is the kernel
 *    specialised for N, one workgroup per tile of 2^T = 2^max(10, r) cells;
 *    "t<T>:<r>/lds" the same with the constant table read from a copy in
 *    LDS; for N = 2^13, 2^14 with more tiles than resident workgroups,
 *    "t<T>:<r>/pipe" runs it on a resident grid whose workgroups load each
 *    next tile while the current one runs; for batches of at most 2^20
 *    transforms, "g<T>:<r>" for every T from
 *    max(10, r) to 14 runs the size-generic persistent kernel of uneven plans
 *    with tiles of 2^T cells over a transform list.
 *  - Uniform plans, N = 2^15, 2^16 (two-pass): "two-pass" (pass A as a
 *    resident grid whose workgroups stride over the tiles, the default) and
 *    "two-pass/all" (one workgroup per tile).
 *  - Uniform plans, N > 2^16 (multi-pass): "multi-pass:f,b,c", the most
 *    forward rounds, backward rounds and chain levels per global pass, for
 *    (f,b,c) in (4,5,5) (the default), (3,5,5), (4,4,5), (4,5,4), (3,4,4),
 *    (5,5,5), with LDS segments of 2^12 cells, and the same six with
 *    segments of 2^13 cells ("multi-pass:f,b,c/s13": one round and one chain
 *    level fewer in the global passes).
 *  - Uneven plans: which tile size serves each transform size of up to 2^14
 *    points, tiles of 2^10 .. 2^14 cells; the assignments for
 *    N <= 2^10, 2^11, 2^12, 2^13, 2^14 of {14,14,14,14,14}, {13,13,13,13,14},
 *    {12,12,12,14,14}, {12,12,12,13,14}, {10,11,12,13,14}, {10,11,12,14,14},
 *    {10,12,12,13,14} (duplicates for the sizes present removed), sizes with
 *    one tile size sharing one launch, each as a resident persistent grid and
 *    as one workgroup per tile ("/all"), and ("/pipe") with every group that
 *    holds only transforms of 2^13 or 2^14 points, more tiles than resident
 *    workgroups, on a resident grid that loads each next tile while the
 *    current one runs; names read "t<T>:<r range>+..".
 *    Schedule 0 runs every transform of up to 2^14 points in ONE persistent
 *    launch.  Longer transforms run after them with the default two-pass or
 *    multi-pass schedule, a run of same-size ones that lie back to back as
 *    one batched exec (its workspace at most 2^22 cells per buffer).
 * A new plan starts on schedule 0, or on the schedule the autotuner chose for
 * a plan of the same shape on the same kind of device, if the schedule cache
 * holds one: a JSON file at $QFT_SCHEDULE_CACHE ("off" disables it), else
 * $XDG_CACHE_HOME/qft-gfx950/schedules.json, else
 * $HOME/.cache/qft-gfx950/schedules.json.  An unreadable file or an entry
 * that names no schedule of the plan is ignored, so the file may be deleted
 * at any time.
 *
 * qft_plan_schedules: number of schedules and the one exec uses.
 * qft_plan_schedule_name: a static description (see above), valid until the
 *   plan is destroyed; NULL for a bad plan or index.
 * qft_plan_set_schedule: selects the schedule exec uses (e.g. a stored
 *   autotuning result); QFT_ERROR_INVALID_VALUE for a bad index.
 * qft_plan_autotune: runs every schedule once to warm up and then `reps`
 *   times (1..10000), timed with HIP events on `stream`, selects the fastest,
 *   returns its index in *chosen (may be NULL) and records it in the schedule
 *   cache (best effort); ms[i], i < ms_len, gets the mean time of schedule i
 *   in milliseconds (ms may be NULL when ms_len = 0).  It overwrites `out`
 *   with F in (in is left unchanged unless in == out), synchronises the
 *   stream and must not be called during graph capture or while another exec
 *   of the plan is in flight.
 */
qft_status qft_plan_schedules(qft_plan_t plan, int* count, int* chosen);
const char* qft_plan_schedule_name(qft_plan_t plan, int schedule);
qft_status qft_plan_set_schedule(qft_plan_t plan, int schedule);
qft_status qft_plan_autotune(qft_plan_t plan, const void* in, void* out, void* stream, int reps,
                             double* ms, int ms_len, int* chosen);

/*
 * Real-input plans (the rdft, dct and dst functions of Sec. 4.2 and Sec.
 * 5.2 as entry points of their own).  `batch` real signals of N = 2^log2n
 * points, 1 <= log2n <= QFT_MAX_LOG2N (up to 2^14 in one workgroup's tile,
 * longer ones through the multi-pass path with a device scratch of
 * 2 * ceil(batch/2) * N complex FP32 values).  Storage:
 * QFT_C32 = FP32 reals (and complex FP32 outputs), QFT_C16 = FP16 (complex
 * FP16 outputs), FP32 arithmetic either way.  Two real signals travel
 * through the transform together, one in each lane of a complex cell, so a
 * real plan costs about half a complex plan of the same batch.  Such a plan
 * serves qft_exec_rdft and qft_exec_dct0_dst0 only; the complex exec and
 * autotune entry points reject it with QFT_ERROR_INVALID_VALUE.
 * qft_plan_info reports total_points = batch*N, algo_bytes = the rdft's
 * read + write, flops_5nlogn = 2.5 N log2 N per signal and flops_actual =
 * 2 N log2 N - 4N + 6 per signal (Table 2, RDFT row).
 */
qft_status qft_plan_create_real(qft_plan_t* plan, int log2n, int64_t batch, qft_dtype dtype,
                                int device);

/*
 * Real-input DFT (rdft, Sec. 4.2): for each real signal x (row b of `in`,
 * batch x N reals, at element b*N) the half spectrum
 *     X(k) = sum_n x(n) exp(-2*pi*i*n*k/N),  k = 0..N/2,
 * (row b of `out`, batch x (N/2 + 1) complex values, at element b*(N/2+1));
 * X(N-k) = conj X(k) gives the rest.  Re X(k) is the DCT-0 of the folded
 * signal c and Im X(k) = -(DST-0 of d).  `in` and `out` must not overlap.
 */
qft_status qft_exec_rdft(qft_plan_t plan, const void* in, void* out, void* stream);

/*
 * DCT-0 and DST-0 of periodization N (dct on s_dc_tt, eq. qft_0B; dst on
 * s_ds_tt, eq. qft_0C):
 *     C(k) = c(0) + (-1)^k c(N/2) + sum_{n=1}^{N/2-1} c(n) cos(2*pi*n*k/N),
 *            k = 0..N/2   (c, C: batch x (N/2 + 1) reals, row b at b*(N/2+1));
 *     S(k) = sum_{n=1}^{N/2-1} d(n) sin(2*pi*n*k/N),
 *            k = 1..N/2-1 (d, S: batch x (N/2 - 1) reals, row b at
 *            b*(N/2-1), d(n) and S(k) at index n-1, k-1).
 * The real fold of Sec. 4.2 (c(n) = x(n) + x(N-n), d(n) = x(n) - x(N-n))
 * turns an rdft into exactly these two.  Either pair (c, C) or (d, S) may be
 * NULL (both members of a pair), not both; for N = 2 the DST-0 is empty and
 * (d, S) are ignored.  c == C and d == S (in place) are allowed; any other
 * overlap of the four ranges gives QFT_ERROR_OVERLAP.
 */
qft_status qft_exec_dct0_dst0(qft_plan_t plan, const void* c, const void* d, void* C, void* S,
                              void* stream);

/*
 * Host-only (no GPU needed): writes the FP32 constant table used for
 * transforms up to N = 2^log2n_max into out[0 .. N/4 - 1].  Entry L + m,
 * for L = 1, 2, 4, .., N/8 and 0 <= m < L, is
 *     1 / (2 cos(pi (2m + 1) / (4L)))
 * (the secant 1/(2 cos(theta n)) of eq. qft_38A with theta = 2*pi/(8L) and
 * odd n = 2m + 1), evaluated in FP64 as 1 / (2 sin(pi (2L - 2m - 1) / (4L)))
 * and rounded once to FP32.  out[0] is 0 (unused).  Entry 1 is
 * 1/(2 cos(pi/4)) = cos(pi/4), the extra constant of Sec. 6.1.
 * Requires 3 <= log2n_max <= QFT_MAX_LOG2N.
 */
qft_status qft_secant_table(float* out, int log2n_max);

/* Static description of a status code. */
const char* qft_status_string(qft_status s);

/*
 * The hipError_t value of the last QFT_ERROR_HIP on this thread (0 if none).
 * It returns the HIP runtime's own code (an int, as hipError_t is), not a
 * qft_status: QFT_ERROR_HIP says that a HIP call failed, this says which
 * error it reported.
 */
int qft_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QFT_H */
