/*
 * ht.h -- C ABI of libht, a Hessenberg-triangular reduction library for AMD
 * MI355X (gfx950).
 *
 * Method: Steel & Vandebril, "Parallel two-stage reduction to
 * Hessenberg-triangular form" (arXiv 2301.07964).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are square, n x n, column major: element (i,j) (0-based) lives at
 *    p[i + j*ld].  Real matrices are double; complex matrices are interleaved
 *    (re, im) pairs of double (C99 double _Complex / hipDoubleComplex layout).
 *  - Matrix pointers are DEVICE pointers (memory from hipMalloc or any
 *    allocator that returns device-accessible memory, e.g. torch).  The caller
 *    owns them; the library never frees or retains them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call validates its arguments on the host, then only ENQUEUES work on
 *    `stream` and returns; results are ready after the stream synchronises.
 *    Calls on different streams may run concurrently; calls that share a
 *    matrix must be ordered by the caller.
 *  - Workspace is taken from a cache inside the library, one per (device,
 *    stream); it grows on demand (hipMalloc, which synchronises the device)
 *    and is reused afterwards.  ht_workspace_bytes() reports the size a call
 *    needs, for admission control by a caller that budgets device memory.
 *  - Return value: 0 = enqueued; -k = argument k is invalid (LAPACK INFO
 *    style, 1-based); > 0 = HT_ERR_* (a HIP failure).  Asynchronous kernel
 *    faults surface at the caller's synchronisation of `stream`.
 *  - Thread safety: calls from several host threads are safe when they use
 *    different streams.
 */
#ifndef HT_H
#define HT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HT_OK 0
#define HT_ERR_HIP 1     /* a HIP runtime call failed */
#define HT_ERR_NOMEM 2   /* device workspace allocation failed */
#define HT_ERR_LAUNCH 3  /* a kernel launch failed */
#define HT_ERR_NOTSUP 4  /* configuration not supported by the library */
#define HT_ERR_TIMEOUT 5 /* a bounded device-side wait gave up (ht_stream_status) */
#define HT_ERR_SCRATCH 6 /* workspace larger than the fixed scratch (ht_stage2_noalloc) */

/*
 * ht_stage2 -- reduce an r-Hessenberg-triangular pencil to Hessenberg-
 * triangular form (stage two; Section 3, unblocked algorithm in the appendix,
 * blocked as generate + apply phases, Section 3.2).
 *
 *   H  (in/out) n x n: on entry r-Hessenberg (H[i,j] = 0 for i > j + r; the
 *      entries below that band are NOT read); on exit upper Hessenberg with
 *      exact zeros below the first subdiagonal.
 *   T  (in/out) n x n: on entry upper triangular (entries below the diagonal
 *      are NOT read); on exit upper triangular with exact zeros below.
 *   Q, Z (in/out) n x n or NULL: on exit Q <- Q*Q2 and Z <- Z*Z2 where
 *      (H_in, T_in) = Q2 (H_out, T_out) Z2^H (pass the identity to obtain Q2,
 *      Z2; pass stage-one factors to obtain the whole reduction).  NULL means
 *      "do not accumulate".
 *   n >= 0, r >= 1 (r >= n-1 is accepted; r == 1 or n <= 2 only writes the
 *      exact zeros), ld >= max(1, n) is shared by the four matrices.
 * Errors: -5 n < 0, -6 r < 1, -7 ld < max(1,n), -1/-2 NULL H/T (n > 0).
 * Reflector conventions: LAPACK xLARFG; left updates use G^H; the opposite
 * reflector is generated from the first row of the RQ orthogonal factor of
 * the current diagonal block of T, normalised to a real positive first
 * nonzero entry.
 */
int ht_stage2(double *H, double *T, double *Q, double *Z,
              int64_t n, int64_t r, int64_t ld, void *stream);

/* Complex128 analogue of ht_stage2 (interleaved re/im doubles). */
int ht_stage2_z(void *H, void *T, void *Q, void *Z,
                int64_t n, int64_t r, int64_t ld, void *stream);

/*
 * ht_stage2_q -- ht_stage2 with an explicit number q of sweeps per delayed
 * update group (Section 3.2).  q = 0 selects the built-in choice.  Requires
 * 1 <= q <= r (else -8).  Used by the autotuner and by tests.
 */
int ht_stage2_q(double *H, double *T, double *Q, double *Z,
                int64_t n, int64_t r, int64_t ld, int64_t q, void *stream);
int ht_stage2_z_q(void *H, void *T, void *Q, void *Z,
                  int64_t n, int64_t r, int64_t ld, int64_t q, void *stream);

/*
 * ht_stage2_noalloc -- ht_stage2 for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, semantics, results and errors as
 * ht_stage2 (same kernels and reflectors), except:
 *   - The workspace comes from a fixed device array of
 *     HT_NOALLOC_SCRATCH_BYTES (64 MiB) that the library holds on every
 *     device it runs on until the process ends; the call allocates nothing
 *     (no hipMalloc/hipFree, no stream or event creation, no library routine
 *     that allocates).  Every size with ht_workspace_bytes(n, r, 0, 0) <=
 *     HT_NOALLOC_SCRATCH_BYTES - 256 fits (n <= 2832 at r = 32, 8398 at
 *     r = 16, 20654 at r = 8; the call takes one of the two reflector buffers
 *     that figure includes, so somewhat larger n fit too); a call that does
 *     not fit returns HT_ERR_SCRATCH and enqueues nothing.
 *   - Every kernel runs on `stream` (Q and Z are not overlapped on a second
 *     stream) and kernel timing (ht_profile_enable) does not apply.
 *   - status: NULL or a DEVICE int owned by the caller; a device-side wait
 *     that gives up ORs 1 into it (the output is then invalid), so the caller
 *     zeroes it before the call and reads it after synchronising `stream`.
 *     With NULL such a failure is not reported.
 *   - Every call on one device shares that device's scratch and overwrites
 *     it: calls that may overlap on one device (different streams, or host
 *     threads) race and must be serialised by the caller.  The scratch keeps
 *     the last call's contents; every counter a call reads is cleared by that
 *     call's own kernels.
 * The first call on a device looks up the device address of its copy of the
 * scratch (hipGetSymbolAddress, no allocation).
 */
#define HT_NOALLOC_SCRATCH_BYTES (64ll << 20)
int ht_stage2_noalloc(double *H, double *T, double *Q, double *Z, int64_t n,
                      int64_t r, int64_t ld, int *status, void *stream);

/*
 * ht_stage2_sweeps -- the first jmax sweeps of stage two only (sweeps
 * j = 1..jmax of the unblocked algorithm, Section 3.1; jmax < 0 or
 * jmax >= n-2 means all of them, i.e. ht_stage2_q).  The sweeps are run in
 * groups of q as ht_stage2_q does, the last group cut at jmax.  On exit
 * columns 1..jmax of H are reduced (exact zeros below the first subdiagonal),
 * the rest of (H, T) holds the band structure the unblocked algorithm leaves
 * after sweep jmax (its structural zeros written as exact zeros), and Q, Z
 * are accumulated as for ht_stage2.  The final exact-zero pass of a complete
 * reduction is not run when jmax < n-2.  Meant for checking a long reduction
 * one prefix at a time, and for callers that reduce a pencil in pieces.
 * Errors as ht_stage2_q.
 */
int ht_stage2_sweeps(double *H, double *T, double *Q, double *Z, int64_t n,
                     int64_t r, int64_t ld, int64_t q, int64_t jmax,
                     void *stream);
int ht_stage2_z_sweeps(void *H, void *T, void *Q, void *Z, int64_t n,
                       int64_t r, int64_t ld, int64_t q, int64_t jmax,
                       void *stream);

/*
 * ht_stream_status -- device-side failures of the calls enqueued on `stream`
 * since the last query.  The generate kernel of stage two coordinates its
 * workgroups with bounded waits on device counters (Section 3.2's pipeline of
 * sweeps); a wait that gives up sets a bit in a per-(device, stream) status
 * word and every workgroup then exits normally, with the output of that call
 * invalid.  This call waits for `stream`, reads and clears that word, and
 * returns 0 (no failure), HT_ERR_TIMEOUT, or HT_ERR_HIP / HT_ERR_NOMEM.
 */
int ht_stream_status(void *stream);

/*
 * Process-wide knobs (defaults in brackets).  ht_set_knob returns 0, -1 for an
 * unknown knob or -2 for a value out of range; ht_get_knob returns the value
 * or -1 for an unknown knob.  Calls already enqueued are not affected.
 *   HT_KNOB_WAIT_POLLS [2^22]: polls before a device-side wait gives up; 0
 *     makes every wait give up at once (used to test the failure path).
 *   HT_KNOB_UPDATE_TILE_ROWS [0]: tiles of 16 rows per wavefront in the
 *     matrix-core right updates; 0 = automatic (2 for n >= 8192), 1 or 2.
 *   HT_KNOB_LOOKAHEAD [1]: lets the generate phase of group g+1 run while
 *     the left updates of group g are still in progress (Section 3.3's
 *     lookahead: each tile of 16 columns of the left pass announces when its
 *     part of the next group's band is final, and the generation waits for
 *     exactly the tiles it reads): 0 never, 1 for n >= 1024, 2 always; real
 *     and complex pencils with r in {4, 8, 16, 32} on the allocating entry
 *     points, while no lookahead call on another stream of the device is
 *     still running (otherwise that call runs its groups in sequence).
 *     The same values switch stage one (ht_rhess*) to its three-stream
 *     schedule (Section 2.3's task split): the Q and Z passes, and each
 *     block's pass over the rows of B that the following block factors do
 *     not read, run on two streams the library keeps beside the caller's
 *     (per device and caller stream); the call is still ordered on the
 *     caller's stream, and its results are bitwise those of the one-stream
 *     schedule.
 */
#define HT_KNOB_WAIT_POLLS 1
#define HT_KNOB_UPDATE_TILE_ROWS 2
#define HT_KNOB_LOOKAHEAD 3
int ht_set_knob(int knob, int64_t value);
int64_t ht_get_knob(int knob);

/*
 * ht_stage2_batched -- `count` independent stage-two reductions (pencils of
 * uneven n and r, each as ht_stage2 defines it) in ONE persistent launch:
 * workgroups (or single wavefronts, per ht_batched_set_tuning) take whole
 * pencils from device-side queues, longest first, and chase their bulges
 * with the unblocked algorithm of the appendix (Section 3.1), each reflector
 * applied at once to its full range.  The reflectors are
 * those of ht_stage2, so the results agree with it up to rounding.  Meant
 * for many small pencils (n up to about a thousand), where the latency of
 * the sweep steps, not flops, bounds the time.
 *   H, T, Q, Z, n, r, ld, q are HOST arrays of length `count`; Q[b] / Z[b]
 *   may be NULL; q may be NULL (q[b] is validated like ht_stage2_q's q and
 *   otherwise unused: the unblocked chase has no group size).  The arrays are
 *   read before the call returns.  The matrices must not overlap.
 * Errors: -1 count < 0, -2..-5 NULL array (or NULL H[b]/T[b] with n[b] > 0),
 * -6 n array, -7 r array, -8 ld array, -9 q array (first offending entry
 * decides); HT_ERR_NOTSUP for min(r, n-1) > 32.
 */
int ht_stage2_batched(int64_t count, double *const *H, double *const *T,
                      double *const *Q, double *const *Z, const int64_t *n,
                      const int64_t *r, const int64_t *ld, const int64_t *q,
                      void *stream);
int ht_stage2_batched_z(int64_t count, void *const *H, void *const *T,
                        void *const *Q, void *const *Z, const int64_t *n,
                        const int64_t *r, const int64_t *ld, const int64_t *q,
                        void *stream);

/*
 * ht_batched_set_tuning -- the table that decides, per pencil, how
 * ht_stage2_batched(_z) reduces it: by a workgroup of 256 threads or by a
 * single wavefront of 64 (four pencils per workgroup at a time).  Entry e
 * applies to pencils with n <= n_max[e] and min(r, n-1) == r[e] (r[e] = 0:
 * any r); the first matching entry decides; threads[e] is 64 or 256.
 * Without a matching entry a pencil with n <= 128 takes a wavefront.  The
 * arrays are host arrays, copied before return; entries = 0 clears the table.
 * Process-wide; calls already enqueued are not affected.  Meant for the
 * autotuner's table (paper_2301_07964_amd/autotune.py).
 * Errors: -1 entries < 0, -2 NULL array, -3 r < 0, -4 threads not 64 or 256.
 */
int ht_batched_set_tuning(int64_t entries, const int64_t *n_max, const int64_t *r,
                          const int64_t *threads);

/*
 * ht_rhess -- stage one: reduce a dense pencil (A, B) to r-Hessenberg-
 * triangular form (Section 2.2, blocked stage-one algorithm in the appendix),
 * after a QR factorisation of B (the experiments of Section 4 replace B by
 * the R factor of its QR).  Panel width n_b = min(r, n-1) <= 32; the blocks
 * of the panel QRs have p*n_b rows (p panel blocks, overlapping by n_b),
 * p = ht_rhess_default_p(n, r) (the largest p <= 8 with p*n_b <= 64, at
 * least 2); ht_rhess_p takes p explicitly (2 <= p, p*n_b <= 64, else -8).
 *   A, B (in/out): dense on entry; on exit A is r-Hessenberg (exact zeros
 *   below the r-th subdiagonal) and B upper triangular (exact zeros below);
 *   Q <- Q*Q1, Z <- Z*Z1 with (A_in, B_in) = Q1 (A_out, B_out) Z1^H, where
 *   Q1 e1 is the first column of the QR factor of B and Z1 e1 = e1.  Q, Z
 *   may be NULL; the four matrices must not overlap.  The output depends
 *   on (n_b, p); the HT form reached after
 *   ht_stage2 does not (up to the unimodular diagonal scaling that the
 *   reflector conventions fix).
 * Errors as ht_stage2 (-5 n, -6 r, -7 ld, -1/-2 NULL A/B, -8 p);
 * HT_ERR_NOTSUP for n_b > 32.
 */
int ht_rhess(double *A, double *B, double *Q, double *Z,
             int64_t n, int64_t r, int64_t ld, void *stream);
int ht_rhess_z(void *A, void *B, void *Q, void *Z,
               int64_t n, int64_t r, int64_t ld, void *stream);
int ht_rhess_p(double *A, double *B, double *Q, double *Z,
               int64_t n, int64_t r, int64_t ld, int64_t p, void *stream);
int ht_rhess_z_p(void *A, void *B, void *Q, void *Z,
                 int64_t n, int64_t r, int64_t ld, int64_t p, void *stream);
/* The built-in p of ht_rhess for (n, r); -1 for n < 0 or r < 1. */
int64_t ht_rhess_default_p(int64_t n, int64_t r);

/*
 * Device workspace (bytes) that a call with these sizes takes from the
 * per-stream cache (is_complex: 0 real, 1 complex; q = 0: built-in choice).
 * Returns -1 for invalid sizes.
 */
int64_t ht_workspace_bytes(int64_t n, int64_t r, int64_t q, int is_complex);

/*
 * Device workspace (bytes) that ht_rhess / ht_rhess_p takes from the
 * per-stream cache (p = 0: built-in choice).  Returns -1 for invalid sizes
 * (including r > 32 or p out of range).
 */
int64_t ht_rhess_workspace_bytes(int64_t n, int64_t r, int64_t p, int is_complex);

/*
 * Grow the workspace cached for (current device, stream) to at least `bytes`
 * now (blocking: an existing smaller buffer is released after the stream has
 * drained).  Later calls on that stream whose workspace fits neither allocate
 * nor synchronise, which keeps a request loop's host thread from stalling
 * when a larger request arrives.  Returns 0, -1 for bytes < 0, or
 * HT_ERR_NOMEM / HT_ERR_HIP.
 */
int ht_reserve_workspace(int64_t bytes, void *stream);

/* Release the calling thread's cached workspaces on the current device. */
void ht_release_workspace(void);

/* The built-in group size q for (n, r). */
int64_t ht_default_q(int64_t n, int64_t r);

/* Static description of an error code (never NULL). */
const char *ht_strerror(int code);

/* Library version string. */
const char *ht_version(void);

/* Diagnostic text of the calling thread's last launch failure ("" if none). */
const char *ht_last_error_message(void);

/*
 * Kernel timing (diagnostics).  ht_profile_enable(1) makes every later call
 * bracket each kernel launch with HIP events recorded on its stream (small
 * overhead).  ht_profile_read() waits for the recorded events, writes the
 * summed milliseconds and the launch counts of each kernel class into
 * ms[0..nclasses-1] / count[0..nclasses-1] (either may be NULL) and forgets
 * the records.  Classes: 0 band copy, 1 generate, 2 right update of H and T,
 * 3 left update of H and T, 4 exact-zero passes, 5 update of Q and Z (runs on
 * a second stream, concurrently with classes 2-4), 6 accumulation of the
 * window factors.  Returns 0 or HT_ERR_HIP.
 */
int ht_profile_enable(int on);
int ht_profile_read(double *ms, int64_t *count, int nclasses);

/*
 * Per-pencil completion times of the calling thread's last ht_stage2_batched
 * call made while kernel timing was enabled: ms[b] = milliseconds from the
 * earliest pencil start of that launch to the completion of pencil b, from the
 * device wall clock.  `count` must equal that call's count.  Waits for the
 * call's stream.  Returns 0, -1 (no such call or count mismatch) or HT_ERR_HIP.
 */
int ht_batched_completion_ms(double *ms, int64_t count);

#ifdef __cplusplus
}
#endif
#endif /* HT_H */
