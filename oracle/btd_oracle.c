/*
 * btd_oracle.c -- plain, slow, FP64 CPU oracle for the decomposition method
 * (DM) of Belov, Nugumanov & Yakovlev, "Decomposition method for
 * block-tridiagonal matrix systems" (arXiv:1505.06864).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, helper or table with the GPU
 * library and includes nothing from it.
 *
 * Notation (the build's letters, which differ from the paper's):
 *   B_i X_{i-1} + A_i X_i + C_i X_{i+1} = F_i,   i = 0..N-1 (0-based rows),
 *   A_i diagonal, B_i sub-diagonal, C_i super-diagonal M x M blocks,
 *   X_i, F_i are M x R blocks.  B_0 and C_{N-1} are never read
 *   (the paper's boundary convention of its problem statement, Sec. 2 Eq. eq01).
 *   P = number of subsystems (the paper's M), M = block size (the paper's n),
 *   R = number of right-hand-side columns (the paper's l).
 *
 * Storage: row-major.  Block i of A/B/C starts at i*M*M; block i of F/X
 * starts at i*M*R and is an M x R row-major tile.
 *
 * What each function follows:
 *   or_inverse      -- block inversion as the paper costs it (Sec. 4): LU with
 *                      partial pivoting, then a solve against the identity.
 *   or_ta_chunk     -- the Thomas algorithm (Sec. 3, forward auxiliaries
 *                      G_i, the paper's script-A_i and script-B_i, then the
 *                      backward stage), with the structural zero-skipping for
 *                      the spike right-hand sides that Sec. 4 counts
 *                      (top-seeded vs bottom-seeded RHS).
 *   or_dm_solve     -- the DM (Sec. 2, Eqs. e220-e232 and endSolution), with
 *                      the coupling system solved by the TA or recursively by
 *                      the DM (Sec. 4.2, Eq. DMrec1).
 *   or_dm_chunk     -- a subsystem solved by the DM itself (recursion into
 *                      the subsystems, Sec. 4.2.2, Eqs. DMrec121-DMrec122).
 *   or_gepp_solve   -- textbook dense Gaussian elimination with partial
 *                      pivoting (first maximum wins), for tiny inputs.
 *   or_residual     -- ||F - A X||_2 / ||F||_2 per RHS column.
 *   or_partition    -- the equal-split separator choice (Sec. 2; equal
 *                      subsystem sizes as in Sec. 5 with the remainder given
 *                      to the first subsystems).
 *   or_default_m    -- number of subsystems of the coupling system for the
 *                      recursive call, Eq. SuppMatrM with its m <= P/3 rule.
 *
 * Every block product and block inversion is counted in the paper's units
 * (Sec. 4): an inversion costs n^3, a product of an n x n block with an
 * n x n block costs n^3, with an n x l block costs n^2 l.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    long long inv; /* block inversions (n^3 each)                          */
    long long mm;  /* block x (n x n) products, incl. applying G_i (n^3)   */
    long long mr;  /* block x (n x l) products (n^2 l each)                */
} or_counter_t;

/* Optional intermediates written by or_dm_solve (any pointer may be NULL).
 * D, E, ZL, ZR are [N][M][M]; y, z are [N][M][R] (chunk rows only);
 * Hd, Hb, Hc are [P-1][M][M]; fhat, h are [P-1][M][R]. */
typedef struct {
    double *D, *E, *ZL, *ZR, *y, *z;
    double *Hd, *Hb, *Hc, *fhat, *h;
} or_aux_t;

/* Status codes (mirrors the meaning, not the code, of the library's). */
#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_SINGULAR 1
#define OR_ERR_NOMEM 2

static void cnt_add(or_counter_t *c, long long inv, long long mm, long long mr) {
    if (!c) return;
#ifdef _OPENMP
#pragma omp atomic
#endif
    c->inv += inv;
#ifdef _OPENMP
#pragma omp atomic
#endif
    c->mm += mm;
#ifdef _OPENMP
#pragma omp atomic
#endif
    c->mr += mr;
}

/* Cp (m x n) = beta * Cp + alpha * Ap (m x k) * Bp (k x n); plain loops,
 * accumulation in the textbook order over k. */
static void mm(int m, int k, int n, double alpha, const double *Ap, int lda,
               const double *Bp, int ldb, double beta, double *Cp, int ldc) {
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int p = 0; p < k; ++p) s += Ap[(size_t)i * lda + p] * Bp[(size_t)p * ldb + j];
            double old = (beta == 0.0) ? 0.0 : beta * Cp[(size_t)i * ldc + j];
            Cp[(size_t)i * ldc + j] = old + alpha * s;
        }
    }
}

/* G = D^{-1}: LU factorisation with partial pivoting (row interchanges,
 * first maximum wins), then forward and back substitution against the
 * columns of the identity (Sec. 4: LU costs n^3/3, the identity solve 2n^3/3).
 * Returns 0, or 1 + column index of an exactly zero pivot. */
int or_inverse(int n, const double *D, double *G) {
    double *lu = (double *)malloc(sizeof(double) * (size_t)n * n);
    int *perm = (int *)malloc(sizeof(int) * (size_t)n);
    if (!lu || !perm) { free(lu); free(perm); return -2; }
    memcpy(lu, D, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    int status = 0;
    for (int j = 0; j < n; ++j) {
        int p = j;
        double best = fabs(lu[(size_t)j * n + j]);
        for (int i = j + 1; i < n; ++i) {
            double v = fabs(lu[(size_t)i * n + j]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) { status = 1 + j; break; }
        if (p != j) {
            for (int c = 0; c < n; ++c) {
                double t = lu[(size_t)j * n + c];
                lu[(size_t)j * n + c] = lu[(size_t)p * n + c];
                lu[(size_t)p * n + c] = t;
            }
            int t = perm[j]; perm[j] = perm[p]; perm[p] = t;
        }
        double piv = lu[(size_t)j * n + j];
        for (int i = j + 1; i < n; ++i) {
            double l = lu[(size_t)i * n + j] / piv;
            lu[(size_t)i * n + j] = l;
            for (int c = j + 1; c < n; ++c) lu[(size_t)i * n + c] -= l * lu[(size_t)j * n + c];
        }
    }
    if (status == 0) {
        /* Solve L U G = Pm I, one column of the identity at a time. */
        double *col = (double *)malloc(sizeof(double) * (size_t)n);
        for (int c = 0; c < n; ++c) {
            for (int i = 0; i < n; ++i) col[i] = (perm[i] == c) ? 1.0 : 0.0;
            for (int i = 0; i < n; ++i) { /* unit lower */
                double s = col[i];
                for (int k = 0; k < i; ++k) s -= lu[(size_t)i * n + k] * col[k];
                col[i] = s;
            }
            for (int i = n - 1; i >= 0; --i) { /* upper */
                double s = col[i];
                for (int k = i + 1; k < n; ++k) s -= lu[(size_t)i * n + k] * col[k];
                col[i] = s / lu[(size_t)i * n + i];
            }
            for (int i = 0; i < n; ++i) G[(size_t)i * n + c] = col[i];
        }
        free(col);
    }
    free(lu);
    free(perm);
    return status;
}

/* Thomas algorithm on one run of nk consecutive block rows (Sec. 3), with up
 * to three kinds of right-hand side solved together as the DM needs (Eq. e231):
 *   F   : full n x R blocks (may be NULL when R == 0);
 *   sL  : an M x M block present only in the first row (left spike seed,
 *         the first block of W_R^k), zero elsewhere; NULL if absent;
 *   sR  : an M x M block present only in the last row (right spike seed),
 *         zero elsewhere; NULL if absent.
 * Products with blocks known to be zero are skipped, which is the structure
 * the paper's operation counts of Sec. 4 assume.
 * Outputs (row-major, nk rows each; NULL to skip): z = solution for F,
 * ZL, ZR = spike solutions.  D and E (if non-NULL) receive the pivot-free
 * intermediates D_i = A_i - B_i E_{i-1} and E_i = D_i^{-1} C_i (i < nk-1).
 * Returns 0, or 1 + local row index of a singular D_i (its column in *bad_col). */
static int or_ta_chunk(int nk, int M, int R, const double *A, const double *B, const double *C,
                       const double *F, const double *sL, const double *sR, double *z, double *ZL,
                       double *ZR, double *Dout, double *Eout, double *yout, or_counter_t *cnt,
                       int *bad_col) {
    const size_t MM = (size_t)M * M, MR = (size_t)M * R;
    double *D = (double *)malloc(sizeof(double) * MM);
    double *G = (double *)malloc(sizeof(double) * MM);
    double *E = (double *)malloc(sizeof(double) * MM * (size_t)(nk > 1 ? nk - 1 : 1));
    double *y = (double *)malloc(sizeof(double) * (MR ? MR : 1) * (size_t)nk);
    double *yL = sL ? (double *)malloc(sizeof(double) * MM * (size_t)nk) : NULL;
    double *yR = sR ? (double *)malloc(sizeof(double) * MM) : NULL;
    double *t = (double *)malloc(sizeof(double) * (MM > MR ? MM : (MR ? MR : 1)));
    int status = 0;
    long long c_inv = 0, c_mm = 0, c_mr = 0;
    for (int i = 0; i < nk; ++i) {
        const double *Ai = A + (size_t)i * MM, *Bi = B + (size_t)i * MM, *Ci = C + (size_t)i * MM;
        /* D_i = A_i - B_i E_{i-1}; G_i = D_i^{-1} */
        memcpy(D, Ai, sizeof(double) * MM);
        if (i > 0) { mm(M, M, M, -1.0, Bi, M, E + (size_t)(i - 1) * MM, M, 1.0, D, M); c_mm++; }
        if (Dout) memcpy(Dout + (size_t)i * MM, D, sizeof(double) * MM);
        int s = or_inverse(M, D, G);
        c_inv++;
        if (s != 0) { status = 1 + i; if (bad_col) *bad_col = s - 1; break; }
        /* E_i = G_i C_i (the paper's script-A_i), rows 0..nk-2 */
        if (i < nk - 1) {
            mm(M, M, M, 1.0, G, M, Ci, M, 0.0, E + (size_t)i * MM, M); c_mm++;
            if (Eout) memcpy(Eout + (size_t)i * MM, E + (size_t)i * MM, sizeof(double) * MM);
        }
        /* y_i = G_i (F_i - B_i y_{i-1}) (the paper's script-B_i) */
        if (R > 0) {
            memcpy(t, F + (size_t)i * MR, sizeof(double) * MR);
            if (i > 0) { mm(M, M, R, -1.0, Bi, M, y + (size_t)(i - 1) * MR, R, 1.0, t, R); c_mr++; }
            mm(M, M, R, 1.0, G, M, t, R, 0.0, y + (size_t)i * MR, R); c_mr++;
            if (yout) memcpy(yout + (size_t)i * MR, y + (size_t)i * MR, sizeof(double) * MR);
        }
        /* left spike: top-seeded, every row carries a nonzero block */
        if (sL) {
            if (i == 0) { mm(M, M, M, 1.0, G, M, sL, M, 0.0, yL, M); c_mm++; }
            else {
                mm(M, M, M, -1.0, Bi, M, yL + (size_t)(i - 1) * MM, M, 0.0, t, M); c_mm++;
                mm(M, M, M, 1.0, G, M, t, M, 0.0, yL + (size_t)i * MM, M); c_mm++;
            }
        }
        /* right spike: bottom-seeded, the forward stage only touches the last row */
        if (sR && i == nk - 1) { mm(M, M, M, 1.0, G, M, sR, M, 0.0, yR, M); c_mm++; }
    }
    if (status == 0) {
        /* backward stage: X_{last} = y_{last}; X_i = y_i - E_i X_{i+1} */
        if (R > 0 && z) {
            memcpy(z + (size_t)(nk - 1) * MR, y + (size_t)(nk - 1) * MR, sizeof(double) * MR);
            for (int i = nk - 2; i >= 0; --i) {
                memcpy(z + (size_t)i * MR, y + (size_t)i * MR, sizeof(double) * MR);
                mm(M, M, R, -1.0, E + (size_t)i * MM, M, z + (size_t)(i + 1) * MR, R, 1.0, z + (size_t)i * MR, R);
                c_mr++;
            }
        }
        if (sL && ZL) {
            memcpy(ZL + (size_t)(nk - 1) * MM, yL + (size_t)(nk - 1) * MM, sizeof(double) * MM);
            for (int i = nk - 2; i >= 0; --i) {
                memcpy(ZL + (size_t)i * MM, yL + (size_t)i * MM, sizeof(double) * MM);
                mm(M, M, M, -1.0, E + (size_t)i * MM, M, ZL + (size_t)(i + 1) * MM, M, 1.0, ZL + (size_t)i * MM, M);
                c_mm++;
            }
        }
        if (sR && ZR) {
            memcpy(ZR + (size_t)(nk - 1) * MM, yR, sizeof(double) * MM);
            for (int i = nk - 2; i >= 0; --i) {
                mm(M, M, M, -1.0, E + (size_t)i * MM, M, ZR + (size_t)(i + 1) * MM, M, 0.0, ZR + (size_t)i * MM, M);
                c_mm++;
            }
        }
        /* The right spike's seed G_last C_last is E at the last row. */
        if (Eout && sR) memcpy(Eout + (size_t)(nk - 1) * MM, yR, sizeof(double) * MM);
    }
    cnt_add(cnt, c_inv, c_mm, c_mr);
    free(D); free(G); free(E); free(y); free(yL); free(yR); free(t);
    return status;
}

int or_partition(int N, int P, int *seps);

/* A subsystem of nk rows solved by the DM itself with J sub-subsystems
 * (recursion into the independent subsystems, Sec. 4.2.2), for the same
 * right-hand sides or_ta_chunk takes: the dense F (R columns), the block sL
 * seeded at the subsystem's first row and the block sR seeded at its last
 * row (either may be NULL).  Writes z, ZL, ZR like or_ta_chunk, for every
 * row of the subsystem.  Zero blocks of the seeded columns are skipped the
 * way the paper counts them (Eqs. DMrec121, DMrec1212, DMrec122): the sL
 * columns enter only the first sub-subsystem (top-seeded there, in place of
 * its missing left spike) and the first row of the inner coupling system;
 * the sR columns only the last sub-subsystem (bottom-seeded, in place of its
 * missing right spike) and the last row of the inner coupling system.  The
 * inner coupling system is solved by the Thomas algorithm.  J < 2, or a
 * subsystem too short for J parts, is the plain Thomas algorithm.
 * Returns 0, or 1 + the failing row within the subsystem. */
static int or_dm_chunk(int nk, int M, int R, const double *A, const double *B, const double *C,
                       const double *F, const double *sL, const double *sR, double *z, double *ZL,
                       double *ZR, int J, or_counter_t *cnt, int *bad_col) {
    if (J < 2 || 2 * J - 1 > nk)
        return or_ta_chunk(nk, M, R, A, B, C, F, sL, sR, z, ZL, ZR, NULL, NULL, NULL, cnt, bad_col);
    const size_t MM = (size_t)M * M, MR = (size_t)M * R;
    const int Jc = J - 1;
    int *sp = (int *)malloc(sizeof(int) * (size_t)Jc);
    or_partition(nk, J, sp);
    /* per row of the subsystem: the inner spikes, the sub-subsystem solution
     * of F, and of the seeded columns (nonzero in the first / last
     * sub-subsystem only) */
    double *iZL = (double *)calloc(MM * (size_t)nk, sizeof(double));
    double *iZR = (double *)calloc(MM * (size_t)nk, sizeof(double));
    double *zf = (double *)calloc(MR * (size_t)nk, sizeof(double));
    double *yL = sL ? (double *)calloc(MM * (size_t)nk, sizeof(double)) : NULL;
    double *yR = sR ? (double *)calloc(MM * (size_t)nk, sizeof(double)) : NULL;
    double *Hd = (double *)calloc(MM * (size_t)Jc, sizeof(double));
    double *Hb = (double *)calloc(MM * (size_t)Jc, sizeof(double));
    double *Hc = (double *)calloc(MM * (size_t)Jc, sizeof(double));
    double *fF = (double *)calloc(MR * (size_t)Jc, sizeof(double));
    double *fL = (double *)calloc(MM, sizeof(double));
    double *fR = (double *)calloc(MM, sizeof(double));
    double *hF = (double *)calloc(MR * (size_t)Jc, sizeof(double));
    double *hL = (double *)calloc(MM * (size_t)Jc, sizeof(double));
    double *hR = (double *)calloc(MM * (size_t)Jc, sizeof(double));
    int status = 0;
    long long c_mm = 0, c_mr = 0;
    /* Eq. e231 within the subsystem: every sub-subsystem by the Thomas
     * algorithm with its own spikes; the outer seeds take the place of the
     * spike a first (last) sub-subsystem does not have */
    for (int i = 0; i < J && !status; ++i) {
        const int r = (i == 0) ? 0 : sp[i - 1] + 1, e = (i == J - 1) ? nk - 1 : sp[i] - 1, n = e - r + 1;
        const double *tL = (i == 0) ? sL : B + (size_t)r * MM;
        const double *tR = (i == J - 1) ? sR : C + (size_t)e * MM;
        double *oL = (i == 0) ? (yL ? yL + (size_t)r * MM : NULL) : iZL + (size_t)r * MM;
        double *oR = (i == J - 1) ? (yR ? yR + (size_t)r * MM : NULL) : iZR + (size_t)r * MM;
        int bc = -1;
        int s = or_ta_chunk(n, M, R, A + (size_t)r * MM, B + (size_t)r * MM, C + (size_t)r * MM, F + (size_t)r * MR,
                            tL, tR, zf + (size_t)r * MR, oL, oR, NULL, NULL, NULL, cnt, &bc);
        if (s) { status = r + s; if (bad_col) *bad_col = bc; }
    }
    if (!status) {
        /* the inner coupling system (Eq. e2311 within the subsystem); the
         * seeded columns' right-hand side has one nonzero block each */
        for (int j = 0; j < Jc; ++j) {
            const int q = sp[j], e = q - 1, r = q + 1;
            const double *Bq = B + (size_t)q * MM, *Cq = C + (size_t)q * MM;
            memcpy(Hd + (size_t)j * MM, A + (size_t)q * MM, sizeof(double) * MM);
            mm(M, M, M, -1.0, Bq, M, iZR + (size_t)e * MM, M, 1.0, Hd + (size_t)j * MM, M); c_mm++;
            mm(M, M, M, -1.0, Cq, M, iZL + (size_t)r * MM, M, 1.0, Hd + (size_t)j * MM, M); c_mm++;
            if (j >= 1) { mm(M, M, M, -1.0, Bq, M, iZL + (size_t)e * MM, M, 0.0, Hb + (size_t)j * MM, M); c_mm++; }
            if (j + 1 <= J - 2) { mm(M, M, M, -1.0, Cq, M, iZR + (size_t)r * MM, M, 0.0, Hc + (size_t)j * MM, M); c_mm++; }
            memcpy(fF + (size_t)j * MR, F + (size_t)q * MR, sizeof(double) * MR);
            mm(M, M, R, -1.0, Bq, M, zf + (size_t)e * MR, R, 1.0, fF + (size_t)j * MR, R); c_mr++;
            mm(M, M, R, -1.0, Cq, M, zf + (size_t)r * MR, R, 1.0, fF + (size_t)j * MR, R); c_mr++;
        }
        if (sL) { mm(M, M, M, -1.0, B + (size_t)sp[0] * MM, M, yL + (size_t)(sp[0] - 1) * MM, M, 0.0, fL, M); c_mm++; }
        if (sR) {
            const int q = sp[Jc - 1];
            mm(M, M, M, -1.0, C + (size_t)q * MM, M, yR + (size_t)(q + 1) * MM, M, 0.0, fR, M); c_mm++;
        }
        /* Eq. e232 within the subsystem by the Thomas algorithm: F columns
         * dense, sL columns seeded at its first row, sR columns at its last */
        int bc = -1;
        int s = or_ta_chunk(Jc, M, R, Hd, Hb, Hc, fF, sL ? fL : NULL, sR ? fR : NULL, hF, sL ? hL : NULL,
                            sR ? hR : NULL, NULL, NULL, NULL, cnt, &bc);
        if (s) { status = sp[s - 1] + 1; if (bad_col) *bad_col = bc; }
    }
    if (!status) {
        /* Eq. endSolution within the subsystem for the three column groups */
        for (int j = 0; j < Jc; ++j) {
            memcpy(z + (size_t)sp[j] * MR, hF + (size_t)j * MR, sizeof(double) * MR);
            if (sL) memcpy(ZL + (size_t)sp[j] * MM, hL + (size_t)j * MM, sizeof(double) * MM);
            if (sR) memcpy(ZR + (size_t)sp[j] * MM, hR + (size_t)j * MM, sizeof(double) * MM);
        }
        for (int i = 0; i < J; ++i) {
            const int r = (i == 0) ? 0 : sp[i - 1] + 1, e = (i == J - 1) ? nk - 1 : sp[i] - 1;
            for (int row = r; row <= e; ++row) {
                const double *zl = iZL + (size_t)row * MM, *zr = iZR + (size_t)row * MM;
                double *zi = z + (size_t)row * MR;
                memcpy(zi, zf + (size_t)row * MR, sizeof(double) * MR);
                if (i > 0) { mm(M, M, R, -1.0, zl, M, hF + (size_t)(i - 1) * MR, R, 1.0, zi, R); c_mr++; }
                if (i < J - 1) { mm(M, M, R, -1.0, zr, M, hF + (size_t)i * MR, R, 1.0, zi, R); c_mr++; }
                if (sL) {
                    double *o = ZL + (size_t)row * MM;
                    memcpy(o, yL + (size_t)row * MM, sizeof(double) * MM);
                    if (i > 0) { mm(M, M, M, -1.0, zl, M, hL + (size_t)(i - 1) * MM, M, 1.0, o, M); c_mm++; }
                    if (i < J - 1) { mm(M, M, M, -1.0, zr, M, hL + (size_t)i * MM, M, 1.0, o, M); c_mm++; }
                }
                if (sR) {
                    double *o = ZR + (size_t)row * MM;
                    memcpy(o, yR + (size_t)row * MM, sizeof(double) * MM);
                    if (i > 0) { mm(M, M, M, -1.0, zl, M, hR + (size_t)(i - 1) * MM, M, 1.0, o, M); c_mm++; }
                    if (i < J - 1) { mm(M, M, M, -1.0, zr, M, hR + (size_t)i * MM, M, 1.0, o, M); c_mm++; }
                }
            }
        }
    }
    cnt_add(cnt, 0, c_mm, c_mr);
    free(sp); free(iZL); free(iZR); free(zf); free(yL); free(yR); free(Hd); free(Hb); free(Hc);
    free(fF); free(fL); free(fR); free(hF); free(hL); free(hR);
    return status;
}

/* Equal-split separators: P-1 rows q_0 < ... < q_{P-2} (0-based), none in
 * the first or the last row, every subsystem non-empty.  Subsystem sizes are
 * floor((N-P+1)/P), the first (N-P+1) mod P subsystems one row longer.
 * Returns 0, or OR_ERR_ARG if P < 1 or 2P-1 > N. */
int or_partition(int N, int P, int *seps) {
    if (P < 1 || N < 1 || (P > 1 && 2 * P - 1 > N)) return OR_ERR_ARG;
    int rows = N - (P - 1), base = rows / P, rem = rows % P, pos = 0;
    for (int k = 0; k < P - 1; ++k) {
        pos += base + (k < rem ? 1 : 0);
        seps[k] = pos;
        pos += 1;
    }
    return OR_OK;
}

/* Subsystem count for the DM applied to the coupling system of P-1 block rows
 * (Eq. SuppMatrM: m = sqrt(P/3 (5 + 2/(1+R/M))) rounded, capped at
 * floor(P/3), at least 2).  Returns 1 (plain TA) when the coupling system has
 * fewer than three block rows. */
int or_default_m(int P, int M, int R) {
    if (P - 1 < 3) return 1;
    double ms = sqrt((double)P / 3.0 * (5.0 + 2.0 / (1.0 + (double)R / (double)M)));
    int m = (int)floor(ms + 0.5);
    if (m > P / 3) m = P / 3;
    if (m < 2) m = 2;
    return m;
}

static int check_seps(int N, int P, const int *seps) {
    int prev = -1;
    for (int k = 0; k < P - 1; ++k) {
        if (seps[k] <= prev + 1 || seps[k] >= N - 1) return OR_ERR_ARG;
        prev = seps[k];
    }
    return OR_OK;
}

/* Plain Thomas algorithm over all N rows (Sec. 3).  X may alias nothing. */
int or_ta_solve(int N, int M, int R, const double *A, const double *B, const double *C,
                const double *F, double *X, or_counter_t *cnt, int *bad_row, int *bad_col) {
    if (N < 1 || M < 1 || R < 1) return OR_ERR_ARG;
    int s = or_ta_chunk(N, M, R, A, B, C, F, NULL, NULL, X, NULL, NULL, NULL, NULL, NULL, cnt, bad_col);
    if (s) { if (bad_row) *bad_row = s - 1; return OR_ERR_SINGULAR; }
    return OR_OK;
}

/* Decomposition method (Sec. 2).  seps: P-1 0-based separator rows or NULL
 * for the equal split; depth: number of DM levels applied to the coupling
 * system (0 = Thomas algorithm, Eq. e232; >= 1 = recursive DM, Eq. DMrec1,
 * with or_default_m subsystems); J >= 2: every subsystem solved by the DM
 * with J equal sub-subsystems (recursion into the subsystems, Sec. 4.2.2;
 * with depth >= 1 both recursions).  P == 1 is the plain Thomas algorithm.
 * nthreads > 0 fixes the OpenMP team for the independent subsystems. */
int or_dm_solve(int N, int M, int R, int P, const int *seps_in, int depth, int J, const double *A,
                const double *B, const double *C, const double *F, double *X, or_aux_t *aux,
                or_counter_t *cnt, int nthreads, int *bad_row, int *bad_col) {
    if (N < 1 || M < 1 || R < 1 || P < 1 || depth < 0 || J < 1) return OR_ERR_ARG;
    const size_t MM = (size_t)M * M, MR = (size_t)M * R;
    if (P == 1) {
        int s = or_ta_chunk(N, M, R, A, B, C, F, NULL, NULL, X, NULL, NULL, aux ? aux->D : NULL,
                            aux ? aux->E : NULL, aux ? aux->y : NULL, cnt, bad_col);
        if (aux && aux->z && s == 0) memcpy(aux->z, X, sizeof(double) * MR * (size_t)N);
        if (s) { if (bad_row) *bad_row = s - 1; return OR_ERR_SINGULAR; }
        return OR_OK;
    }
    if (2 * P - 1 > N) return OR_ERR_ARG;
    int *seps = (int *)malloc(sizeof(int) * (size_t)(P - 1));
    if (seps_in) memcpy(seps, seps_in, sizeof(int) * (size_t)(P - 1));
    else or_partition(N, P, seps);
    if (check_seps(N, P, seps) != OR_OK) { free(seps); return OR_ERR_ARG; }

    /* spikes for every row (only chunk rows are written) */
    double *ZL = (double *)calloc(MM * (size_t)N, sizeof(double));
    double *ZR = (double *)calloc(MM * (size_t)N, sizeof(double));
    double *z = (double *)calloc(MR * (size_t)N, sizeof(double));
    int status = OR_OK, srow = -1, scol = -1;

    /* Eq. e231: independent subsystem solves S^k [z^k | Z^k] = [F_s^k | W_R^k]. */
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int k = 0; k < P; ++k) {
        int r = (k == 0) ? 0 : seps[k - 1] + 1;
        int e = (k == P - 1) ? N - 1 : seps[k] - 1;
        int nk = e - r + 1;
        const double *sL = (k > 0) ? B + (size_t)r * MM : NULL;     /* couples to h^{k-1} */
        const double *sR = (k < P - 1) ? C + (size_t)e * MM : NULL; /* couples to h^k     */
        int bc = -1;
        int s = (J >= 2)
                    ? or_dm_chunk(nk, M, R, A + (size_t)r * MM, B + (size_t)r * MM, C + (size_t)r * MM,
                                  F + (size_t)r * MR, sL, sR, z + (size_t)r * MR, ZL + (size_t)r * MM,
                                  ZR + (size_t)r * MM, J, cnt, &bc)
                    : or_ta_chunk(nk, M, R, A + (size_t)r * MM, B + (size_t)r * MM, C + (size_t)r * MM,
                                  F + (size_t)r * MR, sL, sR, z + (size_t)r * MR, ZL + (size_t)r * MM,
                                  ZR + (size_t)r * MM, aux && aux->D ? aux->D + (size_t)r * MM : NULL,
                                  aux && aux->E ? aux->E + (size_t)r * MM : NULL,
                                  aux && aux->y ? aux->y + (size_t)r * MR : NULL, cnt, &bc);
        if (s) {
#ifdef _OPENMP
#pragma omp critical
#endif
            { if (status == OR_OK || r + s - 1 < srow) { status = OR_ERR_SINGULAR; srow = r + s - 1; scol = bc; } }
        }
    }
    if (aux && aux->ZL) memcpy(aux->ZL, ZL, sizeof(double) * MM * (size_t)N);
    if (aux && aux->ZR) memcpy(aux->ZR, ZR, sizeof(double) * MM * (size_t)N);
    if (aux && aux->z) memcpy(aux->z, z, sizeof(double) * MR * (size_t)N);
    if (status != OR_OK) {
        if (bad_row) *bad_row = srow;
        if (bad_col) *bad_col = scol;
        free(seps); free(ZL); free(ZR); free(z);
        return status;
    }

    /* Eq. e2311: coupling matrix H - W_L S^{-1} W_R and vector F_h - W_L S^{-1} F_s.
     * Separator j (row q) sits between subsystem j (last row e) and j+1 (first row r). */
    const int Pc = P - 1;
    double *Hd = (double *)calloc(MM * (size_t)Pc, sizeof(double));
    double *Hb = (double *)calloc(MM * (size_t)Pc, sizeof(double));
    double *Hc = (double *)calloc(MM * (size_t)Pc, sizeof(double));
    double *fh = (double *)calloc(MR * (size_t)Pc, sizeof(double));
    double *h = (double *)calloc(MR * (size_t)Pc, sizeof(double));
    long long c_mm = 0, c_mr = 0;
    for (int j = 0; j < Pc; ++j) {
        int q = seps[j], e = q - 1, r = q + 1;
        const double *Bq = B + (size_t)q * MM, *Cq = C + (size_t)q * MM;
        memcpy(Hd + (size_t)j * MM, A + (size_t)q * MM, sizeof(double) * MM);
        /* subsystem j: its right spike always exists (j < P-1) */
        mm(M, M, M, -1.0, Bq, M, ZR + (size_t)e * MM, M, 1.0, Hd + (size_t)j * MM, M); c_mm++;
        if (j >= 1) { mm(M, M, M, -1.0, Bq, M, ZL + (size_t)e * MM, M, 0.0, Hb + (size_t)j * MM, M); c_mm++; }
        /* subsystem j+1: its left spike always exists (j+1 >= 1) */
        mm(M, M, M, -1.0, Cq, M, ZL + (size_t)r * MM, M, 1.0, Hd + (size_t)j * MM, M); c_mm++;
        if (j + 1 <= P - 2) { mm(M, M, M, -1.0, Cq, M, ZR + (size_t)r * MM, M, 0.0, Hc + (size_t)j * MM, M); c_mm++; }
        memcpy(fh + (size_t)j * MR, F + (size_t)q * MR, sizeof(double) * MR);
        mm(M, M, R, -1.0, Bq, M, z + (size_t)e * MR, R, 1.0, fh + (size_t)j * MR, R); c_mr++;
        mm(M, M, R, -1.0, Cq, M, z + (size_t)r * MR, R, 1.0, fh + (size_t)j * MR, R); c_mr++;
    }
    cnt_add(cnt, 0, c_mm, c_mr);
    if (aux && aux->Hd) memcpy(aux->Hd, Hd, sizeof(double) * MM * (size_t)Pc);
    if (aux && aux->Hb) memcpy(aux->Hb, Hb, sizeof(double) * MM * (size_t)Pc);
    if (aux && aux->Hc) memcpy(aux->Hc, Hc, sizeof(double) * MM * (size_t)Pc);
    if (aux && aux->fhat) memcpy(aux->fhat, fh, sizeof(double) * MR * (size_t)Pc);

    /* Eq. e232: the supplementary block-tridiagonal system of P-1 rows, by the
     * TA or, for depth >= 1, by the DM itself (Eq. DMrec1). */
    int m = (depth > 0) ? or_default_m(P, M, R) : 1;
    int sb = -1, sc = -1;
    int s = or_dm_solve(Pc, M, R, m, NULL, depth > 0 ? depth - 1 : 0, 1, Hd, Hb, Hc, fh, h, NULL, cnt,
                        nthreads, &sb, &sc);
    if (s != OR_OK) {
        if (bad_row) *bad_row = (sb >= 0 && sb < Pc) ? seps[sb] : -1;
        if (bad_col) *bad_col = sc;
        status = s;
    } else {
        if (aux && aux->h) memcpy(aux->h, h, sizeof(double) * MR * (size_t)Pc);
        /* Eq. endSolution: s^k = z^k - Z_L^k h^{k-1} - Z_R^k h^k, h^0 = h^P = 0. */
        for (int j = 0; j < Pc; ++j) memcpy(X + (size_t)seps[j] * MR, h + (size_t)j * MR, sizeof(double) * MR);
        long long r_mr = 0;
        for (int k = 0; k < P; ++k) {
            int r = (k == 0) ? 0 : seps[k - 1] + 1;
            int e = (k == P - 1) ? N - 1 : seps[k] - 1;
            for (int i = r; i <= e; ++i) {
                double *Xi = X + (size_t)i * MR;
                memcpy(Xi, z + (size_t)i * MR, sizeof(double) * MR);
                if (k > 0) { mm(M, M, R, -1.0, ZL + (size_t)i * MM, M, h + (size_t)(k - 1) * MR, R, 1.0, Xi, R); r_mr++; }
                if (k < P - 1) { mm(M, M, R, -1.0, ZR + (size_t)i * MM, M, h + (size_t)k * MR, R, 1.0, Xi, R); r_mr++; }
            }
        }
        cnt_add(cnt, 0, 0, r_mr);
    }
    free(seps); free(ZL); free(ZR); free(z); free(Hd); free(Hb); free(Hc); free(fh); free(h);
    return status;
}

/* Textbook dense Gaussian elimination with partial pivoting on an n x n
 * row-major matrix (first maximum wins on ties), nrhs right-hand sides.
 * Returns 0, or 1 + column of an exactly zero pivot. */
int or_gepp_solve(int n, int nrhs, const double *Ad, const double *Bd, double *Xd) {
    double *a = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *b = (double *)malloc(sizeof(double) * (size_t)n * nrhs);
    memcpy(a, Ad, sizeof(double) * (size_t)n * n);
    memcpy(b, Bd, sizeof(double) * (size_t)n * nrhs);
    int status = 0;
    for (int j = 0; j < n && !status; ++j) {
        int p = j;
        double best = fabs(a[(size_t)j * n + j]);
        for (int i = j + 1; i < n; ++i)
            if (fabs(a[(size_t)i * n + j]) > best) { best = fabs(a[(size_t)i * n + j]); p = i; }
        if (best == 0.0) { status = 1 + j; break; }
        if (p != j) {
            for (int c = 0; c < n; ++c) { double t = a[(size_t)j * n + c]; a[(size_t)j * n + c] = a[(size_t)p * n + c]; a[(size_t)p * n + c] = t; }
            for (int c = 0; c < nrhs; ++c) { double t = b[(size_t)j * nrhs + c]; b[(size_t)j * nrhs + c] = b[(size_t)p * nrhs + c]; b[(size_t)p * nrhs + c] = t; }
        }
        for (int i = j + 1; i < n; ++i) {
            double l = a[(size_t)i * n + j] / a[(size_t)j * n + j];
            for (int c = j; c < n; ++c) a[(size_t)i * n + c] -= l * a[(size_t)j * n + c];
            for (int c = 0; c < nrhs; ++c) b[(size_t)i * nrhs + c] -= l * b[(size_t)j * nrhs + c];
        }
    }
    if (!status) {
        for (int c = 0; c < nrhs; ++c)
            for (int i = n - 1; i >= 0; --i) {
                double s = b[(size_t)i * nrhs + c];
                for (int k = i + 1; k < n; ++k) s -= a[(size_t)i * n + k] * Xd[(size_t)k * nrhs + c];
                Xd[(size_t)i * nrhs + c] = s / a[(size_t)i * n + i];
            }
    }
    free(a); free(b);
    return status;
}

/* r = F - (B X_{i-1} + A X_i + C X_{i+1}); out[c] = ||r[:,c]||_2 / ||F[:,c]||_2
 * (out[c] = ||r[:,c]||_2 when F[:,c] = 0). */
void or_residual(int N, int M, int R, const double *A, const double *B, const double *C,
                 const double *X, const double *F, double *out) {
    const size_t MM = (size_t)M * M, MR = (size_t)M * R;
    double *rn = (double *)calloc((size_t)R, sizeof(double));
    double *fn = (double *)calloc((size_t)R, sizeof(double));
    for (int i = 0; i < N; ++i) {
        for (int a = 0; a < M; ++a) {
            for (int c = 0; c < R; ++c) {
                double s = F[(size_t)i * MR + (size_t)a * R + c];
                fn[c] += s * s;
                for (int b = 0; b < M; ++b) {
                    s -= A[(size_t)i * MM + (size_t)a * M + b] * X[(size_t)i * MR + (size_t)b * R + c];
                    if (i > 0) s -= B[(size_t)i * MM + (size_t)a * M + b] * X[(size_t)(i - 1) * MR + (size_t)b * R + c];
                    if (i < N - 1) s -= C[(size_t)i * MM + (size_t)a * M + b] * X[(size_t)(i + 1) * MR + (size_t)b * R + c];
                }
                rn[c] += s * s;
            }
        }
    }
    for (int c = 0; c < R; ++c) out[c] = fn[c] > 0.0 ? sqrt(rn[c]) / sqrt(fn[c]) : sqrt(rn[c]);
    free(rn); free(fn);
}

/* Threads the OpenMP runtime would use (1 without OpenMP). */
int or_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
