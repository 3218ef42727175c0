/*
 * btd.h -- C ABI of the MI355X (gfx950) decomposition-method solver for
 * block-tridiagonal systems (Belov, Nugumanov & Yakovlev,
 * "Decomposition method for block-tridiagonal matrix systems",
 * arXiv:1505.06864).
 *
 * The system (Sec. 2, Eq. eq01, written here with A diagonal, B
 * sub-diagonal and C super-diagonal, which are the paper's C, A and B):
 *
 *     B_i X_{i-1} + A_i X_i + C_i X_{i+1} = F_i,    i = 0 .. N-1,
 *
 * with M x M blocks A_i, B_i, C_i and M x R blocks X_i, F_i.  B_0 and C_{N-1}
 * are never read.
 *
 * Method (Sec. 2): P-1 separator block rows split the other rows into P
 * subsystems.  Each subsystem is eliminated independently by the block
 * Thomas algorithm (Sec. 3; here block LU with partial pivoting inside
 * every diagonal block, triangular solves and Schur-complement products),
 * which yields its part z of the solution and its two spikes Z_L, Z_R
 * (Eq. e231).  The coupling system of P-1 block rows (Eqs. e2311, e232) is
 * solved by the Thomas algorithm or, when depth >= 1, by the same method
 * applied recursively (Sec. 4.2, Eq. DMrec1).  The subsystem rows are then
 * recovered as X = z - Z_L h^{k-1} - Z_R h^k (Eq. endSolution).
 *
 * Conventions for every entry point:
 *   - Matrix and vector pointers are DEVICE pointers (HBM of the current
 *     HIP device), FP64, row-major.  A, B, C: [N][M][M] (block i at
 *     offset i*M*M).  F, X: [N][M][R] (block row i is an M x R row-major
 *     tile at offset i*M*R).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All work is enqueued asynchronously on that stream; the calls return
 *     once the work is enqueued.
 *   - The library never allocates device memory.  The caller provides the
 *     workspaces, sized by btd_workspace_bytes, and keeps them alive.
 *   - Return value 0 = enqueued.  A negative value -k means that argument k
 *     (1-based position in the call) is invalid; it is detected on the host
 *     before anything is enqueued, and nothing is enqueued then.
 *     BTD_ERR_LAUNCH means a HIP launch failed (work enqueued before it may
 *     still run).  Numerical failures are found on the device and read back
 *     with btd_get_info after the stream has been synchronised.
 *   - Calls on one plan are not thread-safe.  Distinct plans may be used
 *     from distinct host threads on distinct streams: every call orders its
 *     own work with events of the calling thread, so no call waits on
 *     another call's stream.  The library's side streams (at most four per
 *     device, created once) are shared by all threads, so concurrent calls
 *     are correct but their side-stream launches interleave in issue order.
 */
#ifndef BTD_H
#define BTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (btd_get_info, btd_status_string, call returns). */
#define BTD_OK 0
#define BTD_ERR_SINGULAR 1   /* an exactly zero pivot in the LU of a diagonal block D_i */
#define BTD_ERR_NONFINITE 2  /* a pivot that is NaN or infinite                          */
#define BTD_ERR_LAUNCH 3     /* a HIP launch or copy failed (returned by the call)       */
#define BTD_ERR_SCRATCH 4    /* btd_solve_noalloc: the solve needs more than the static scratch */
#define BTD_ERR_NOT_CONVERGED 5 /* btd_solve_refine: the tolerance was not reached             */

#define BTD_PREC_F64 0
/* Mixed precision: the block products of the factor sweeps of the top level
 * (the Schur complements D_i = A_i - B_i E_{i-1} and the spike products)
 * run on FP32 MFMA with FP32 accumulation; everything is stored in FP64, and
 * the LU of D_i, the coupling systems, every solve, the residual and the
 * correction stay FP64.  btd_solve then gives about FP32 accuracy;
 * btd_solve_refine reaches FP64 accuracy by iterative refinement. */
#define BTD_PREC_F32_REFINE 1

/* Largest block size the kernels accept (diagonal-block LU panel held in LDS). */
#define BTD_MAX_M 512

typedef struct btd_plan_s *btd_plan_t;

/*
 * Problem description.
 *   N         block rows, N >= 1.
 *   M         block size, 1 <= M <= BTD_MAX_M.
 *   P         number of subsystems, 1 <= P and 2P-1 <= N when P > 1
 *             (every subsystem keeps at least one row; Sec. 2 places the
 *             separators anywhere from the second to the next-to-last row).
 *             P = 1 is the plain block Thomas algorithm (Sec. 3).
 *   depth     DM levels applied to the coupling system (0 = Thomas
 *             algorithm, Eq. e232; d >= 1 = DM with m subsystems, Eq.
 *             DMrec1, m from Eq. SuppMatrM: m = round(sqrt(P/3 (5 + 2/(1 +
 *             R/M)))) capped at floor(P/3), at least 2; levels whose
 *             coupling system has fewer than 3 rows use the Thomas
 *             algorithm).  R here is max_nrhs.
 *   prec      BTD_PREC_F64 or BTD_PREC_F32_REFINE.
 *   max_nrhs  largest R a later btd_solve may use (>= 1).
 *   seps      NULL for the equal split (subsystem sizes floor((N-P+1)/P),
 *             the first (N-P+1) mod P subsystems one row longer), or a HOST
 *             array of P-1 strictly increasing 0-based separator rows with
 *             1 <= q, q <= N-2 and at least one row between neighbours.
 *             Copied during btd_factor; not retained.
 *   coupling_rows  how the coupling systems of the recursion levels are
 *             split: 0 = m from Eq. SuppMatrM as described under depth (the
 *             choice that minimises the operation count of Sec. 5); k >= 1 =
 *             subsystems of about k rows, m = floor((Nc + 1) / (k + 1)) for a
 *             coupling system of Nc rows (at least 2; the Thomas algorithm
 *             when Nc < 3).  Small k trades extra operations for fewer
 *             sequential steps, which is what bounds a recursion level on a
 *             GPU.
 *   sub_parts J: 0 or 1 = off; J >= 2 = recursion into the subsystems
 *             (Sec. 4.2.2): every one of the P subsystems is itself solved by
 *             the method with J equal sub-subsystems (each subsystem needs
 *             at least 2J-1 rows).  Realised as one level of P*J subsystems
 *             (the P-1 separators plus J-1 inner separators per subsystem,
 *             equal split inside each subsystem) whose coupling system is
 *             split at the P-1 outer separators: its P subsystems are the
 *             subsystems' own coupling systems (J-1 rows each), and its
 *             coupling system is the outer one (P-1 rows; the Schur
 *             complement onto the separators, the same matrix the plain
 *             method forms), solved according to depth and coupling_rows
 *             (depth >= 1: both recursions, Sec. 4.2.3).  The solution is
 *             the same; the intermediate spikes of whole subsystems are not
 *             formed.
 */
typedef struct {
    int32_t N, M, P, depth, prec, max_nrhs;
    const int32_t *seps;
    int32_t coupling_rows;
    int32_t sub_parts;
} btd_desc_t;

/*
 * Workspace sizes in bytes for a description.  factor_ws holds the LU
 * factors, pivots, E_i = D_i^{-1} C_i, the spikes and the coupling
 * system(s); it lives as long as the plan.  solve_ws is scratch for one
 * btd_solve (or btd_solve_batch) call with up to max_nrhs columns.
 * Returns 0 or -1 (invalid description).  Either output pointer may be NULL.
 */
int btd_workspace_bytes(const btd_desc_t *desc, size_t *factor_ws, size_t *solve_ws);

/*
 * Factor (Sec. 2 steps up to and including the coupling-system factor):
 * for every subsystem the block LU of D_i = A_i - B_i E_{i-1}, E_i and both
 * spikes; the coupling matrix H - W_L S^{-1} W_R (Eq. e2311) and its own
 * factorisation.  A, B, C are BORROWED by the plan (btd_residual and later
 * solves read them): keep them unchanged and allocated until
 * btd_plan_destroy.  factor_ws (>= factor bytes, 256-byte aligned) is
 * owned by the plan until btd_plan_destroy.  *out receives a host-side plan
 * handle (a small host allocation).
 * Returns 0; -1 invalid description or seps; -2/-3/-4 NULL A/B/C; -5 NULL or
 * not 256-byte-aligned factor_ws; -6 factor_bytes too small; -8 NULL out;
 * BTD_ERR_LAUNCH.
 */
int btd_factor(const btd_desc_t *desc, const double *A, const double *B, const double *C,
               void *factor_ws, size_t factor_bytes, void *stream, btd_plan_t *out);

/*
 * btd_factor and then btd_solve of nrhs columns (1 <= nrhs <= max_nrhs) in
 * one call, with the same plan, results and ownership as those two calls.
 * The difference is the schedule: each recursion level's right-hand-side
 * sweep and coupling right-hand side (Eqs. e231, e2311) need only that
 * level's forward-sweep factors, so they run on a library side stream
 * while the level's spikes (Eq. e232) and the deeper levels are still
 * being factored; the recoveries (Eq. endSolution) follow on `stream`.
 * The side stream is forked from and joined back to `stream`, so the call
 * is ordered on `stream` like any other (and may be captured in a graph).
 * Without side streams it runs the two steps one after the other.
 * F, X, solve_ws as for btd_solve (X may equal F); factor_ws and *out as
 * for btd_factor.
 * Returns 0; -1..-6 and -8 as btd_factor; -7 nrhs out of range; -9/-10
 * NULL F/X; -11 NULL or misaligned solve_ws; -12 solve_bytes too small;
 * BTD_ERR_LAUNCH.  On an error no plan is returned.
 */
int btd_factor_solve(const btd_desc_t *desc, const double *A, const double *B, const double *C,
                     void *factor_ws, size_t factor_bytes, int32_t nrhs, const double *F, double *X,
                     void *solve_ws, size_t solve_bytes, void *stream, btd_plan_t *out);

/*
 * Solve with a factored plan (Sec. 2, Eqs. e231 (RHS part), e2311 (vector
 * part), e232, endSolution): X = A^{-1} F for nrhs columns,
 * 1 <= nrhs <= max_nrhs.  F and X are [N][M][nrhs]; X may equal F (in
 * place).  solve_ws (>= solve bytes, 256-byte aligned) is scratch for the
 * duration of the call on `stream`.
 * Returns 0; -1 NULL plan; -2 nrhs out of range; -3/-4 NULL F/X; -5 NULL or
 * misaligned solve_ws; -6 solve_bytes too small; BTD_ERR_LAUNCH.
 */
int btd_solve(btd_plan_t plan, int32_t nrhs, const double *F, double *X, void *solve_ws,
              size_t solve_bytes, void *stream);

/*
 * Solve several factored systems in one call: for s < count,
 * X[s] = A_s^{-1} F[s] with nrhs[s] columns.  plans, nrhs, F, X are HOST
 * arrays of length count (F[s], X[s] device pointers).  solve_ws must be at
 * least the largest solve size of the plans; with room for k such solves
 * (each rounded up to 256 bytes), up to k of them (at most 4) run side by side on the
 * library's side streams, each in its own slice of solve_ws, forked from and
 * joined back to `stream`; otherwise they run one after another on `stream`.
 * Results do not depend on which: every solve is the same computation.
 * Entries must not share an X array.
 * Returns 0; -1 count < 0 or a NULL array; -(1000 + s) for the first bad
 * entry s (NULL plan or pointer, nrhs out of range); -6 NULL, misaligned or
 * too small solve_ws; BTD_ERR_LAUNCH.
 */
int btd_solve_batch(int32_t count, const btd_plan_t *plans, const int32_t *nrhs,
                    const double *const *F, double *const *X, void *solve_ws, size_t solve_bytes,
                    void *stream);

/*
 * Iterative refinement (for BTD_PREC_F32_REFINE plans; any plan works):
 *   X = solve(F); then while max_c ||F - A X||_2 / ||F||_2 > tol and fewer
 *   than max_iter corrections were made: D = solve(F - A X), X += D,
 * with the residual F - A X and the correction X += D in FP64 against the
 * plan's FP64 blocks A, B, C.  BLOCKING: the residual norms are read on the
 * host after every residual (the call synchronises `stream` each time), so
 * it cannot be captured in a graph.  work (>= btd_refine_work_bytes, 256-byte
 * aligned) holds the solve workspace, the residual vector and the norms.
 * *iters (may be NULL) = corrections made; *resid (may be NULL) = the final
 * max_c relative residual.  X must not alias F.
 * Returns 0 when the final residual is <= tol; BTD_ERR_NOT_CONVERGED when
 * it is not after max_iter corrections (X holds the last iterate);
 * -1 NULL plan; -2 nrhs out of range; -3/-4 NULL F/X or X == F; -5 NULL or
 * misaligned work; -6 work too small; -7 tol not positive or max_iter < 0;
 * BTD_ERR_LAUNCH.
 */
size_t btd_refine_work_bytes(btd_plan_t plan, int32_t nrhs);
int btd_solve_refine(btd_plan_t plan, int32_t nrhs, const double *F, double *X, void *work, size_t work_bytes,
                     double tol, int32_t max_iter, int32_t *iters, double *resid, void *stream);

/*
 * btd_solve without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The same computation and kernels as
 * btd_solve; its scratch (the coupling right-hand sides of every recursion
 * level) is a static device array of BTD_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device it runs on until the process ends.  The call
 * allocates nothing.  Every call on one device shares that device's array:
 * calls that overlap on one device (two streams, or two host threads) race
 * and give wrong results; serialise them.  The array keeps the last call's
 * contents, none of which a later call reads before writing it.
 * Returns 0; -1 NULL plan; -2 nrhs out of range; -3/-4 NULL F/X;
 * BTD_ERR_SCRATCH when btd_workspace_bytes' solve size for this plan and
 * nrhs exceeds BTD_NOALLOC_SCRATCH_BYTES (nothing is enqueued; use btd_solve);
 * BTD_ERR_LAUNCH.
 */
#define BTD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int btd_solve_noalloc(btd_plan_t plan, int32_t nrhs, const double *F, double *X, void *stream);

/*
 * The two halves of btd_solve, for a caller that solves the coupling system
 * itself (for instance with the coupling blocks of btd_plan_level_arrays,
 * or sharded over several devices):
 *
 * btd_solve_local: the per-subsystem part (Sec. 2, Eq. e231 for the
 * right-hand side, and the vector part of Eq. e2311).  Writes z, the
 * solution of every subsystem with its right-hand side F alone, into the
 * subsystem rows of X (separator rows of X are left untouched), and the
 * coupling right-hand side f_j = F_q - B_q z_{q-1} - C_q z_{q+1} of every
 * separator q = q_j into Fhat, a DEVICE array [P-1][M][nrhs] (level 0
 * sizes).  With P = 1 it is the whole solve and Fhat is not used (may be
 * NULL).  X may equal F.
 * btd_solve_finish: given the coupling solution h ([P-1][M][nrhs], DEVICE;
 * may be the Fhat array solved in place) and X from btd_solve_local,
 * writes X_q = h_j at the separators and recovers the subsystem rows,
 * X_i = z_i - Z_L[i] h_{k-1} - Z_R[i] h_k (Eq. endSolution).
 * Neither needs a workspace.  Both return 0; -1 NULL plan; -2 nrhs out of
 * range; -3/-4 NULL F/X (finish: -3 NULL H when P > 1, -4 NULL X); -5 NULL
 * Fhat when P > 1; BTD_ERR_LAUNCH.  btd_solve_local also records the
 * right-hand-side check of btd_get_solve_info.
 */
int btd_solve_local(btd_plan_t plan, int32_t nrhs, const double *F, double *X, double *Fhat, void *stream);
int btd_solve_finish(btd_plan_t plan, int32_t nrhs, const double *H, double *X, void *stream);

/*
 * Status of the right-hand side of the last btd_solve, btd_solve_local or
 * btd_solve_batch entry of `plan`; call after synchronising its stream.
 * Every solve first checks F: *status = BTD_ERR_NONFINITE when F holds a
 * NaN or an infinity, with *block_row = the first such block row i and
 * *col = its right-hand-side column (the smallest (row, column) pair);
 * BTD_OK and -1, -1 otherwise.  Any output pointer may be NULL.  Performs a
 * blocking device-to-host copy.  Returns 0, -1 for a NULL plan, or
 * BTD_ERR_LAUNCH.
 */
int btd_get_solve_info(btd_plan_t plan, int32_t *status, int32_t *block_row, int32_t *col);

/*
 * Read-only device views of one recursion level of a factored plan (level 0
 * = the caller's system; level l >= 1 = the coupling system of level l-1,
 * whose blocks are Hd, Hb, Hc of that level).  For inspection and for
 * callers that build on the intermediates of Sec. 2:
 *   N, M, P   sizes of the level's system and its subsystem count;
 *   A, B, C   the level's blocks ([N][M][M]);
 *   W         [N][M][2M]: columns 0..M-1 of row i hold E_i = D_i^{-1} C_i
 *             (the forward auxiliary of Sec. 3; at the last row of a
 *             subsystem with a right spike it is the spike's seed D^{-1} C,
 *             and it is not defined at the last row of the last subsystem);
 *             columns M..2M-1 hold the forward sweep Y of the left spike in
 *             subsystems k >= 1 (Eq. e231);
 *   Z         [N][M][2M]: [Z_L | Z_R], the spikes of Eq. e231 at subsystem
 *             rows (Z_L defined for k >= 1, Z_R for k <= P-2); NULL when P = 1;
 *   Hd, Hb, Hc  [P-1][M][M]: diagonal, sub- and super-diagonal blocks of the
 *             coupling system (Eq. e2311); NULL when P = 1;
 *   sep       [P+1] device ints: -1, the P-1 separator rows, N.
 * The arrays live in the plan's factor workspace and are valid after the
 * factor's stream has been synchronised and until the next btd_factor into
 * the same workspace.  Returns 0, or -1 for a NULL plan or output, or a
 * level past the last.
 */
typedef struct {
    int32_t N, M, P;
    const double *A, *B, *C;
    const double *W, *Z;
    const double *Hd, *Hb, *Hc;
    const int32_t *sep;
} btd_level_arrays_t;
int btd_plan_level_arrays(btd_plan_t plan, int32_t level, btd_level_arrays_t *out);

/*
 * Relative residual per column (the check of a solve; not a step of the
 * paper): out[c] = ||F[:,c] - (A X)[:,c]||_2 / ||F[:,c]||_2, or the
 * unscaled norm when F[:,c] = 0.  A, B, C, X, F are device pointers, out is
 * a DEVICE array of R doubles, work a DEVICE array of at least
 * btd_residual_work_bytes(N, M, R) bytes.
 * Returns 0; -1 bad sizes; -k for the first NULL pointer argument k
 * (4..10); BTD_ERR_LAUNCH.
 */
size_t btd_residual_work_bytes(int32_t N, int32_t M, int32_t R);
int btd_residual(int32_t N, int32_t M, int32_t R, const double *A, const double *B, const double *C,
                 const double *X, const double *F, double *out, void *work, void *stream);

/*
 * Numerical status of the last btd_factor of `plan`; call after
 * synchronising the factor's stream.  *status = BTD_OK, BTD_ERR_SINGULAR or
 * BTD_ERR_NONFINITE; *block_row = 0-based row i of the first failing D_i
 * (a separator row when the failure was in the coupling system), *col = its
 * pivot column; both -1 when OK.  Any output pointer may be NULL.  Performs
 * a blocking device-to-host copy.  Returns 0, -1 for a NULL plan, or
 * BTD_ERR_LAUNCH when the copy fails.
 */
int btd_get_info(btd_plan_t plan, int32_t *status, int32_t *block_row, int32_t *col);

/* Separator rows of the P subsystems actually used (P-1 entries into a host
 * array; with sub_parts the outer separators only). Returns 0 or -1. */
int btd_plan_separators(btd_plan_t plan, int32_t *seps_out);

/* Subsystem count used for the system at recursion level `level` (level 0 =
 * the top system: P, or P * sub_parts; level l + 1 = the coupling system of
 * level l).  Returns the count, or -1 past the last level. */
int btd_plan_level_parts(btd_plan_t plan, int32_t level);

/* Host-only helpers (no device work): the equal-split separator rows for
 * (N, P) written into seps_out[P-1], and the subsystem count the recursive
 * coupling solve uses for P subsystems, block size M and R columns (Eq.
 * SuppMatrM rule described for btd_desc_t::depth; 1 = Thomas algorithm).
 * Both return -1 for invalid sizes. */
int btd_default_separators(int32_t N, int32_t P, int32_t *seps_out);
/* Host-only: the balanced partition of Sec. 5.1 (Eq. SpeedupMPNk, second case of the speedup
 * analysis): the first and the last subsystem alpha and beta times as long
 * as the middle ones, whose common size is (N - (P-1)) / (P - 2 + alpha +
 * beta), so that on one processor per subsystem the end subsystems (which
 * have one spike fewer) take as long as the middle ones; the paper's values
 * for few right-hand sides are alpha = 7/4, beta = 7/6.  Sizes are rounded
 * to whole rows (first alpha x and last beta x to the nearest row, the rest
 * split evenly over the middle subsystems, the first of them one row longer
 * when it does not divide), every subsystem at least one row.  Writes
 * seps_out[P-1] (0-based separator rows, for btd_desc_t::seps); returns 0,
 * or -1 for invalid sizes or alpha, beta outside [1, 64]. */
int btd_balanced_separators(int32_t N, int32_t P, double alpha, double beta, int32_t *seps_out);
int btd_default_coupling_parts(int32_t P, int32_t M, int32_t R);
/* Subsystem count of the coupling system of a level with P subsystems for a
 * given coupling_rows (see btd_desc_t; 0 gives btd_default_coupling_parts).
 * Returns -1 for invalid sizes. */
int btd_coupling_parts(int32_t P, int32_t M, int32_t R, int32_t coupling_rows);

/*
 * Kernel timing for measurements: while a class is enabled, every launch of
 * that kernel class (on the process's plans, any stream) is bracketed by a
 * pair of HIP events recorded on the launch's stream.  btd_profile_read
 * waits for the recorded events, returns the summed elapsed milliseconds and
 * the number of launches since the last read, and keeps the events for
 * later launches (a measured pass after the first creates no events).
 * Classes: see BTD_KC_*.  btd_profile_enable(-1) disables.  The record is
 * process-wide (guarded by a lock).  Returns 0, or -1 for an unknown class.
 */
#define BTD_KC_FWD_GEMM 0     /* D_i = A_i - B_i E_{i-1} and the left-spike product       */
#define BTD_KC_GETRF 1        /* LU with partial pivoting of D_i                          */
#define BTD_KC_GETRS_FACTOR 2 /* [E_i | Y_i] = D_i^{-1} [C_i | -B_i Y_{i-1}]               */
#define BTD_KC_BWD_GEMM 3     /* backward sweep of the spikes                              */
#define BTD_KC_COUPLE 4       /* coupling matrix assembly (Eq. e2311)                      */
#define BTD_KC_RHS_SWEEP 5    /* per-chunk forward and backward sweep of the right-hand side */
#define BTD_KC_COUPLE_RHS 6   /* coupling right-hand side (Eq. e2311)                      */
#define BTD_KC_RECOVER 7      /* X = z - Z_L h^{k-1} - Z_R h^k (Eq. endSolution)           */
#define BTD_KC_RESIDUAL 8     /* residual check                                            */
#define BTD_KC_DIAG_PREP 9    /* inverses of the 32x32 diagonal blocks of L and U, scaled off-diagonal blocks */
#define BTD_KC_COUNT 10
int btd_profile_enable(int32_t kernel_class);
int btd_profile_read(double *total_ms, int64_t *launches);

/* Releases the host handle.  The caller then owns factor_ws and A, B, C
 * again; enqueued work that uses them must have finished first. */
void btd_plan_destroy(btd_plan_t plan);

/* Static string for a status or argument-error code. */
const char *btd_status_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* BTD_H */
