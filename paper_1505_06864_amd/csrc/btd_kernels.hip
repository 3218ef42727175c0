// btd_kernels.hip -- gfx950 kernels of the decomposition method (DM) for
// block-tridiagonal systems, arXiv:1505.06864.
//
// Notation: B_i X_{i-1} + A_i X_i + C_i X_{i+1} = F_i (A diagonal, B sub-,
// C super-diagonal M x M blocks; the paper's C, A, B of Sec. 2 Eq. eq01).
//
// Per subsystem (chunk) the block Thomas algorithm of Sec. 3 is run with LU
// factors instead of explicit inverses:
//   D_i = A_i - B_i E_{i-1}          (Schur-complement GEMM, FP64 MFMA)
//   P_i D_i = L_i U_i                (blocked LU, wavefront pivot search)
//   [E_i | Y_i] = D_i^{-1} [C_i | -B_i Y_{i-1}]   (TRSM, MFMA updates)
// where Y is the forward sweep of the left spike (seeded by B at the first
// chunk row) and E at the last chunk row is the right-spike seed
// (Eq. e231).  The backward sweep gives the spikes Z = [Z_L | Z_R]; the
// coupling system of Eq. e2311 is assembled from the spike tips; the
// solution follows Eq. endSolution.
//
// All kernels of one step are batched over the chunks (grid.y); the chunk
// map sep[] (sep[0] = -1, sep[k] = separator row of chunk k-1/k, sep[P] = N)
// is read on the device, so every launch has the same shape for any
// partition.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "btd_internal.h"

typedef double v4d __attribute__((ext_vector_type(4)));

namespace btd {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int chunk_first(const Level& L, int k) { return L.sep[k] + 1; }
__device__ __forceinline__ int chunk_last(const Level& L, int k) { return L.sep[k + 1] - 1; }

__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Record a numerical failure; the smallest (level, row, col, code) key wins,
// so the report is independent of scheduling.
__device__ void report_status(unsigned long long* st, int level, int row, int col, int code) {
    unsigned long long key = ((unsigned long long)(level & 0xff) << 56) |
                             ((unsigned long long)(row & 0xffffff) << 32) |
                             ((unsigned long long)(col & 0xffffff) << 8) | (unsigned long long)(code & 0xff);
    atomicMin(st, key);
}

// ------------------------------------------------------------------ GEMM jobs
//
// One job: Out (m x n) = Cin + alpha * (A1 * B1 + A2 * B2), with optional
// extra tile copy CopyOut = CopyIn over the same m x n tile coordinates.
struct Job {
    const double *A1, *B1, *A2, *B2, *Cin, *CopyIn;
    double *Out, *CopyOut;
    int lda1, ldb1, lda2, ldb2, ldc, ldo, ldci, ldco;
    int m, n, k1, k2;
    double alpha;
};

__device__ __forceinline__ void job_clear(Job& j) {
    j.A1 = j.B1 = j.A2 = j.B2 = j.Cin = j.CopyIn = nullptr;
    j.Out = j.CopyOut = nullptr;
    j.lda1 = j.ldb1 = j.lda2 = j.ldb2 = j.ldc = j.ldo = j.ldci = j.ldco = 0;
    j.m = j.n = j.k1 = j.k2 = 0;
    j.alpha = -1.0;
}

// Decode the job of (mode, batch item, part).  Returns false when the
// (batch, part) pair has nothing to do at this step.
template <int MODE>
__device__ bool make_job(const KArgs& ka, int b, int part, Job& j) {
    const Level& L = ka.L;
    const int M = L.M;
    const size_t MM = (size_t)M * M;
    const int M2 = 2 * M;
    job_clear(j);
    j.m = M;
    j.n = M;
    if (MODE == GM_FWD) {
        // chunk b, step t: D_i = A_i - B_i E_{i-1} (part 0, plus C_i -> W_i[:, :M]);
        // Y_i = -B_i Y_{i-1} (part 1, chunks with a left spike).
        const int k = b, t = ka.step;
        const int r = chunk_first(L, k), e = chunk_last(L, k);
        if (t > e - r) return false;
        const int i = r + t;
        if (part == 0) {
            j.Out = L.LU + i * MM; j.ldo = M;
            j.Cin = L.A + i * MM; j.ldc = M;
            if (t > 0) { j.A1 = L.B + i * MM; j.lda1 = M; j.B1 = L.W + (i - 1) * MM * 2; j.ldb1 = M2; j.k1 = M; }
            if (i != L.N - 1) { j.CopyIn = L.C + i * MM; j.ldci = M; j.CopyOut = L.W + i * MM * 2; j.ldco = M2; }
            return true;
        }
        if (k == 0) return false;
        j.Out = L.W + i * MM * 2 + M; j.ldo = M2;
        if (t == 0) { j.Cin = L.B + i * MM; j.ldc = M; }
        else { j.A1 = L.B + i * MM; j.lda1 = M; j.B1 = L.W + (i - 1) * MM * 2 + M; j.ldb1 = M2; j.k1 = M; }
        return true;
    } else if (MODE == GM_BWD) {
        // chunk b, backward step s (row i = e - s): Z_L (part 0, k > 0), Z_R (part 1, k < P-1)
        const int k = b, s = ka.step;
        const int r = chunk_first(L, k), e = chunk_last(L, k);
        if (s > e - r) return false;
        const int i = e - s;
        const double* Wi = L.W + i * MM * 2;
        if (part == 0) {
            if (k == 0) return false;
            j.Out = L.Z + i * MM * 2; j.ldo = M2;
            j.Cin = Wi + M; j.ldc = M2;
            if (s > 0) { j.A1 = Wi; j.lda1 = M2; j.B1 = L.Z + (i + 1) * MM * 2; j.ldb1 = M2; j.k1 = M; }
            return true;
        }
        if (k == L.P - 1) return false;
        j.Out = L.Z + i * MM * 2 + M; j.ldo = M2;
        if (s == 0) { j.Cin = Wi; j.ldc = M2; }
        else { j.A1 = Wi; j.lda1 = M2; j.B1 = L.Z + (i + 1) * MM * 2 + M; j.ldb1 = M2; j.k1 = M; }
        return true;
    } else if (MODE == GM_COUPLE) {
        // separator b at row q between chunk b (last row q-1) and chunk b+1 (first row q+1)
        const int jj = b, q = L.sep[jj + 1];
        const int e = q - 1, r = q + 1;
        const double* Bq = L.B + q * MM;
        const double* Cq = L.C + q * MM;
        if (part == 0) {
            j.Out = L.Hb + jj * MM; j.ldo = M;
            if (jj >= 1) { j.A1 = Bq; j.lda1 = M; j.B1 = L.Z + e * MM * 2; j.ldb1 = M2; j.k1 = M; }
        } else if (part == 1) {
            j.Out = L.Hd + jj * MM; j.ldo = M;
            j.Cin = L.A + q * MM; j.ldc = M;
            j.A1 = Bq; j.lda1 = M; j.B1 = L.Z + e * MM * 2 + M; j.ldb1 = M2; j.k1 = M;
            j.A2 = Cq; j.lda2 = M; j.B2 = L.Z + r * MM * 2; j.ldb2 = M2; j.k2 = M;
        } else {
            j.Out = L.Hc + jj * MM; j.ldo = M;
            if (jj + 1 <= L.P - 2) { j.A1 = Cq; j.lda1 = M; j.B1 = L.Z + r * MM * 2 + M; j.ldb1 = M2; j.k1 = M; }
        }
        return true;
    } else if (MODE == GM_RHS_FWD) {
        const int k = b, t = ka.step, R = ka.R;
        const int r = chunk_first(L, k), e = chunk_last(L, k);
        if (t > e - r) return false;
        const int i = r + t;
        const size_t MR = (size_t)M * R;
        j.n = R;
        j.Out = ka.X + i * MR; j.ldo = R;
        j.Cin = ka.F + i * MR; j.ldc = R;
        if (t > 0) { j.A1 = L.B + i * MM; j.lda1 = M; j.B1 = ka.X + (i - 1) * MR; j.ldb1 = R; j.k1 = M; }
        return true;
    } else if (MODE == GM_RHS_BWD) {
        const int k = b, s = ka.step, R = ka.R;
        const int r = chunk_first(L, k), e = chunk_last(L, k);
        if (s < 1 || s > e - r) return false;
        const int i = e - s;
        const size_t MR = (size_t)M * R;
        j.n = R;
        j.Out = ka.X + i * MR; j.ldo = R;
        j.Cin = ka.X + i * MR; j.ldc = R;
        j.A1 = L.W + i * MM * 2; j.lda1 = M2; j.B1 = ka.X + (i + 1) * MR; j.ldb1 = R; j.k1 = M;
        return true;
    } else if (MODE == GM_COUPLE_RHS) {
        const int jj = b, q = L.sep[jj + 1], R = ka.R;
        const size_t MR = (size_t)M * R;
        j.n = R;
        j.Out = ka.Fc + jj * MR; j.ldo = R;
        j.Cin = ka.F + q * MR; j.ldc = R;
        j.A1 = L.B + q * MM; j.lda1 = M; j.B1 = ka.X + (q - 1) * MR; j.ldb1 = R; j.k1 = M;
        j.A2 = L.C + q * MM; j.lda2 = M; j.B2 = ka.X + (q + 1) * MR; j.ldb2 = R; j.k2 = M;
        return true;
    } else if (MODE == GM_RECOVER) {
        // batch item = block row i; chunk rows: X_i -= Z_L h^{k-1} + Z_R h^k, separators: X_q = h
        const int i = b, R = ka.R, P = L.P;
        const size_t MR = (size_t)M * R;
        int lo = 0, hi = P;  // find k with sep[k] <= i < sep[k+1]  (sep[0] = -1, sep[P] = N)
        while (hi - lo > 1) { int mid = (lo + hi) >> 1; if (L.sep[mid] <= i) lo = mid; else hi = mid; }
        const int k = lo;
        j.n = R;
        j.Out = ka.X + i * MR; j.ldo = R;
        if (L.sep[k] == i) { j.Cin = ka.Fc + (k - 1) * MR; j.ldc = R; return true; }
        j.Cin = ka.X + i * MR; j.ldc = R;
        const double* Zi = L.Z + i * MM * 2;
        if (k > 0 && k < P - 1) { j.A1 = Zi; j.lda1 = M2; j.B1 = ka.Fc + (k - 1) * MR; j.ldb1 = R; j.k1 = M2; }
        else if (k == 0) { j.A1 = Zi + M; j.lda1 = M2; j.B1 = ka.Fc; j.ldb1 = R; j.k1 = M; }
        else { j.A1 = Zi; j.lda1 = M2; j.B1 = ka.Fc + (size_t)(P - 2) * MR; j.ldb1 = R; j.k1 = M; }
        return true;
    }
    return false;
}

// ------------------------------------------------------------------ GEMM tile
//
// 64 x 64 output tile per 256-thread workgroup; wave w owns the 32 x 32
// quadrant (w >> 1, w & 1) as 2 x 2 tiles of v_mfma_f64_16x16x4f64.
// MFMA operand layout (lane l): A element (row l&15, k l>>4); B element
// (k l>>4, col l&15); D holds rows (l>>4)+4*v, col l&15 in register v.
// LDS: As[16][64+AP] (k-major, transposed), Bs[16][64+BP].
constexpr int TB = 64, KB = 16, AP = 4, BP = 4;

__device__ __forceinline__ void load_tiles(const double* __restrict__ A, int lda, const double* __restrict__ Bm,
                                           int ldb, int row0, int col0, int k0, int m, int n, int K, double ra[4],
                                           double rb[4]) {
    const int tid = threadIdx.x;
    {
        const int rr = tid >> 2, kq = (tid & 3) * 4;
        const int gr = row0 + rr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gk = k0 + kq + q;
            ra[q] = (gr < m && gk < K) ? A[(size_t)gr * lda + gk] : 0.0;
        }
    }
    {
        const int kk = tid >> 4, cq = (tid & 15) * 4;
        const int gk = k0 + kk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gc = col0 + cq + q;
            rb[q] = (gk < K && gc < n) ? Bm[(size_t)gk * ldb + gc] : 0.0;
        }
    }
}

__device__ __forceinline__ void store_tiles(double* As, double* Bs, const double ra[4], const double rb[4]) {
    const int tid = threadIdx.x;
    {
        const int rr = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) As[(kq + q) * (TB + AP) + rr] = ra[q];
    }
    {
        const int kk = tid >> 4, cq = (tid & 15) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) Bs[kk * (TB + BP) + cq + q] = rb[q];
    }
}

__device__ void tile_accumulate(const double* __restrict__ A, int lda, const double* __restrict__ Bm, int ldb,
                                int K, int row0, int col0, int m, int n, v4d acc[2][2], double* As, double* Bs) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    double ra[4], rb[4];
    if (K <= 0) return;
    load_tiles(A, lda, Bm, ldb, row0, col0, 0, m, n, K, ra, rb);
    for (int k0 = 0; k0 < K; k0 += KB) {
        __syncthreads();
        store_tiles(As, Bs, ra, rb);
        __syncthreads();
        if (k0 + KB < K) load_tiles(A, lda, Bm, ldb, row0, col0, k0 + KB, m, n, K, ra, rb);
#pragma unroll
        for (int kk = 0; kk < KB / 4; ++kk) {
            const int krow = kk * 4 + (lane >> 4);
            double a0 = As[krow * (TB + AP) + wr + (lane & 15)];
            double a1 = As[krow * (TB + AP) + wr + 16 + (lane & 15)];
            double b0 = Bs[krow * (TB + BP) + wc + (lane & 15)];
            double b1 = Bs[krow * (TB + BP) + wc + 16 + (lane & 15)];
            acc[0][0] = mfma4(a0, b0, acc[0][0]);
            acc[0][1] = mfma4(a0, b1, acc[0][1]);
            acc[1][0] = mfma4(a1, b0, acc[1][0]);
            acc[1][1] = mfma4(a1, b1, acc[1][1]);
        }
    }
}

template <int MODE, int NPARTS>
__global__ __launch_bounds__(256) void k_gemm(const KArgs ka, int tiles_m, int tiles_n) {
    __shared__ double As[KB * (TB + AP)];
    __shared__ double Bs[KB * (TB + BP)];
    const int b = blockIdx.y;
    int bx = blockIdx.x;
    const int tn = bx % tiles_n; bx /= tiles_n;
    const int tm = bx % tiles_m; bx /= tiles_m;
    const int part = bx;
    Job j;
    if (!make_job<MODE>(ka, b, part, j)) return;
    const int row0 = tm * TB, col0 = tn * TB;
    if (row0 >= j.m || col0 >= j.n) return;
    v4d acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = (v4d){0.0, 0.0, 0.0, 0.0};
    tile_accumulate(j.A1, j.lda1, j.B1, j.ldb1, j.k1, row0, col0, j.m, j.n, acc, As, Bs);
    tile_accumulate(j.A2, j.lda2, j.B2, j.ldb2, j.k2, row0, col0, j.m, j.n, acc, As, Bs);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = row0 + (w >> 1) * 32, wc = col0 + (w & 1) * 32;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int col = wc + 16 * c + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wr + 16 * a + (lane >> 4) + 4 * v;
                if (row < j.m && col < j.n) {
                    double base = j.Cin ? j.Cin[(size_t)row * j.ldc + col] : 0.0;
                    j.Out[(size_t)row * j.ldo + col] = base + j.alpha * acc[a][c][v];
                    if (j.CopyOut) j.CopyOut[(size_t)row * j.ldco + col] = j.CopyIn[(size_t)row * j.ldci + col];
                }
            }
        }
}

// ------------------------------------------------------------------ LU
//
// One workgroup (256 threads) per diagonal block D_i: right-looking blocked
// LU with partial pivoting (row interchanges; ties go to the lowest row).
// Panel of NB columns held in LDS (column-major, pitch M+1); the pivot
// search is a per-thread scan, a 64-lane shuffle argmax inside each wave and
// a 4-entry combine across waves.  Row interchanges are applied to the
// columns outside the panel and U12 = L11^{-1} A12 by one thread per column;
// the trailing update A22 -= L21 U12 runs on FP64 MFMA in 32 x 32 wave tiles.
// Epilogue: the permutation (row r of P D is row perm[r] of D) and the
// inverses of the 16 x 16 diagonal blocks of L and U for the solves.
constexpr int NB = 16;

__global__ __launch_bounds__(256) void k_getrf(const KArgs ka) {
    const Level& L = ka.L;
    const int k = blockIdx.x, t = ka.step;
    const int r = chunk_first(L, k), e = chunk_last(L, k);
    if (t > e - r) return;
    const int i = r + t;
    const int M = L.M, PM = M + 1;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double* a = L.LU + (size_t)i * M * M;
    extern __shared__ double sm[];
    double* pan = sm;                       // [NB][M+1]
    double* us = pan + NB * PM;             // [NB][M]
    double* redv = us + NB * M;             // [4]
    int* redi = (int*)(redv + 4);           // [4]
    int* swp = redi + 4;                    // [NB]
    int* sperm = swp + NB;                  // [M]

    for (int rr = tid; rr < M; rr += 256) sperm[rr] = rr;
    int fail_code = 0, fail_col = -1;
    for (int j0 = 0; j0 < M; j0 += NB) {
        const int nb = min(NB, M - j0), h = M - j0;
        __syncthreads();
        for (int idx = tid; idx < h * nb; idx += 256) {
            const int rr = idx / nb, c = idx - rr * nb;
            pan[c * PM + rr] = a[(size_t)(j0 + rr) * M + j0 + c];
        }
        __syncthreads();
        for (int jj = 0; jj < nb; ++jj) {
            double* colj = pan + jj * PM;
            double bv = -1.0;
            int bi = 0x7fffffff;
            for (int rr = jj + tid; rr < h; rr += 256) {
                const double v = fabs(colj[rr]);
                if (v > bv) { bv = v; bi = rr; }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int oi = __shfl_xor(bi, off);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if (lane == 0) { redv[w] = bv; redi[w] = bi; }
            __syncthreads();
            bv = redv[0]; bi = redi[0];
#pragma unroll
            for (int q = 1; q < 4; ++q)
                if (redv[q] > bv || (redv[q] == bv && redi[q] < bi)) { bv = redv[q]; bi = redi[q]; }
            const int p = (bi == 0x7fffffff) ? jj : bi;
            if (p != jj)
                for (int c = tid; c < nb; c += 256) {
                    const double tmp = pan[c * PM + jj];
                    pan[c * PM + jj] = pan[c * PM + p];
                    pan[c * PM + p] = tmp;
                }
            if (tid == 0) {
                swp[jj] = p;
                if (p != jj) { const int tmp = sperm[j0 + jj]; sperm[j0 + jj] = sperm[j0 + p]; sperm[j0 + p] = tmp; }
            }
            __syncthreads();
            const double piv = colj[jj];
            if (fail_code == 0) {
                if (bi == 0x7fffffff || !isfinite(piv)) { fail_code = BTD_ERR_NONFINITE_; fail_col = j0 + jj; }
                else if (piv == 0.0) { fail_code = BTD_ERR_SINGULAR_; fail_col = j0 + jj; }
            }
            if (piv != 0.0) {
                for (int rr = jj + 1 + tid; rr < h; rr += 256) {
                    const double l = colj[rr] / piv;
                    colj[rr] = l;
                    for (int c = jj + 1; c < nb; ++c) pan[c * PM + rr] -= l * pan[c * PM + jj];
                }
            }
            __syncthreads();
        }
        for (int idx = tid; idx < h * nb; idx += 256) {
            const int rr = idx / nb, c = idx - rr * nb;
            a[(size_t)(j0 + rr) * M + j0 + c] = pan[c * PM + rr];
        }
        // row interchanges outside the panel; U12 = L11^{-1} A12
        for (int col = tid; col < M; col += 256) {
            if (col >= j0 && col < j0 + nb) continue;
            for (int jj = 0; jj < nb; ++jj) {
                const int p = swp[jj];
                if (p != jj) {
                    const double tmp = a[(size_t)(j0 + jj) * M + col];
                    a[(size_t)(j0 + jj) * M + col] = a[(size_t)(j0 + p) * M + col];
                    a[(size_t)(j0 + p) * M + col] = tmp;
                }
            }
            if (col >= j0 + nb) {
                double u[NB];
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) {
                    if (jj < nb) {
                        double s = a[(size_t)(j0 + jj) * M + col];
#pragma unroll
                        for (int c = 0; c < jj; ++c) s -= pan[c * PM + jj] * u[c];
                        u[jj] = s;
                        a[(size_t)(j0 + jj) * M + col] = s;
                        us[jj * M + (col - j0 - nb)] = s;
                    } else {
                        u[jj] = 0.0;
                    }
                }
            }
        }
        __syncthreads();
        // trailing update A22 -= L21 U12 on MFMA
        const int mt = h - nb;
        if (mt > 0) {
            const int t32 = (mt + 31) / 32;
            double* a22 = a + (size_t)(j0 + nb) * M + j0 + nb;
            for (int tile = w; tile < t32 * t32; tile += 4) {
                const int tr = (tile / t32) * 32, tc = (tile % t32) * 32;
                v4d acc[2][2];
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y) {
                        const int col = tc + 16 * y + (lane & 15);
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = tr + 16 * x + (lane >> 4) + 4 * v;
                            acc[x][y][v] = (row < mt && col < mt) ? a22[(size_t)row * M + col] : 0.0;
                        }
                    }
#pragma unroll
                for (int kk = 0; kk < NB / 4; ++kk) {
                    const int kr = kk * 4 + (lane >> 4);
                    double av[2], bv2[2];
#pragma unroll
                    for (int x = 0; x < 2; ++x) {
                        const int row = tr + 16 * x + (lane & 15);
                        av[x] = (kr < nb && row < mt) ? -pan[kr * PM + nb + row] : 0.0;
                    }
#pragma unroll
                    for (int y = 0; y < 2; ++y) {
                        const int col = tc + 16 * y + (lane & 15);
                        bv2[y] = (kr < nb && col < mt) ? us[kr * M + col] : 0.0;
                    }
#pragma unroll
                    for (int x = 0; x < 2; ++x)
#pragma unroll
                        for (int y = 0; y < 2; ++y) acc[x][y] = mfma4(av[x], bv2[y], acc[x][y]);
                }
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y) {
                        const int col = tc + 16 * y + (lane & 15);
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = tr + 16 * x + (lane >> 4) + 4 * v;
                            if (row < mt && col < mt) a22[(size_t)row * M + col] = acc[x][y][v];
                        }
                    }
            }
        }
    }
    __syncthreads();
    int* perm = L.perm + (size_t)i * M;
    for (int rr = tid; rr < M; rr += 256) perm[rr] = sperm[rr];
    // inverses of the 16 x 16 diagonal blocks of L (unit lower) and U
    const int nblk = (M + 15) / 16;
    double* di = L.DI + (size_t)i * nblk * 512;
    for (int idx = tid; idx < nblk * 16; idx += 256) {
        const int bb = idx >> 4, jc = idx & 15, b0 = bb * 16, bs = min(16, M - b0);
        double x[16];
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            double s = (rr == jc) ? 1.0 : 0.0;
            if (rr > jc && rr < bs) {
#pragma unroll
                for (int c = 0; c < rr; ++c)
                    if (c >= jc) s -= a[(size_t)(b0 + rr) * M + b0 + c] * x[c];
            }
            x[rr] = s;
        }
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) di[bb * 512 + rr * 16 + jc] = x[rr];
        double y[16];
#pragma unroll
        for (int rr = 15; rr >= 0; --rr) {
            double s;
            if (rr >= bs) s = (rr == jc) ? 1.0 : 0.0;
            else if (rr > jc) s = 0.0;
            else {
                s = (rr == jc) ? 1.0 : 0.0;
#pragma unroll
                for (int c = 15; c > rr; --c)
                    if (c <= jc && c < bs) s -= a[(size_t)(b0 + rr) * M + b0 + c] * y[c];
                s /= a[(size_t)(b0 + rr) * M + b0 + rr];
            }
            y[rr] = s;
        }
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) di[bb * 512 + 256 + rr * 16 + jc] = y[rr];
    }
    if (tid == 0 && fail_code != 0) {
        // the failing row is reported as a row of the system this level solves
        report_status(ka.status, L.level, i, fail_col, fail_code);
    }
}

// ------------------------------------------------------------------ triangular solves
//
// In place on an M x ncols right-hand side (row-major, leading dimension
// ld): X := U^{-1} L^{-1} (P X), one slab of SW columns per workgroup held
// in LDS.  Both sweeps go by 16-row blocks: X_b := inv(T_bb) X_b with the
// inverted diagonal block, then the remaining rows are updated with the
// off-diagonal panel on MFMA.  Column validity is decided per column, so a
// slab can straddle the E and Y halves of W.
template <int SW>
__device__ void getrs_slab(const double* __restrict__ lu, const double* __restrict__ di,
                           const int* __restrict__ perm, double* X, int ld, int M, int c0, int ncols, int valid_lo,
                           int valid_hi, int valid2_lo, int valid2_hi, double* xs) {
    constexpr int PX = SW + 2;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nblk = (M + 15) / 16, Mp = nblk * 16;
    auto valid = [&](int col) {
        return col < ncols && ((col >= valid_lo && col < valid_hi) || (col >= valid2_lo && col < valid2_hi));
    };
    for (int idx = tid; idx < Mp * SW; idx += 256) {
        const int rr = idx / SW, c = idx - rr * SW, col = c0 + c;
        xs[rr * PX + c] = (rr < M && valid(col)) ? X[(size_t)perm[rr] * ld + col] : 0.0;
    }
    __syncthreads();
    constexpr int NSUB = SW / 16;
    // forward: unit lower
    for (int bb = 0; bb < nblk; ++bb) {
        const int b0 = bb * 16;
        // X_b := invL_b X_b   (waves 0..NSUB-1, one 16-column subtile each)
        if (w < NSUB) {
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            const double* il = di + bb * 512;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int kr = kk * 4 + (lane >> 4);
                acc = mfma4(il[(lane & 15) * 16 + kr], xs[(b0 + kr) * PX + w * 16 + (lane & 15)], acc);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int v = 0; v < 4; ++v) xs[(b0 + (lane >> 4) + 4 * v) * PX + w * 16 + (lane & 15)] = acc[v];
        }
        __syncthreads();
        const int nstrip = nblk - bb - 1;
        for (int job = w; job < nstrip * NSUB; job += 4) {
            const int st = job / NSUB, sub = job - st * NSUB;
            const int row0 = b0 + 16 + st * 16, col = sub * 16 + (lane & 15);
            v4d acc;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = xs[(row0 + (lane >> 4) + 4 * v) * PX + col];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int kr = kk * 4 + (lane >> 4);
                const int grow = row0 + (lane & 15), gk = b0 + kr;
                const double av = (grow < M && gk < M) ? -lu[(size_t)grow * M + gk] : 0.0;
                acc = mfma4(av, xs[(b0 + kr) * PX + col], acc);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) xs[(row0 + (lane >> 4) + 4 * v) * PX + col] = acc[v];
        }
        __syncthreads();
    }
    // backward: upper
    for (int bb = nblk - 1; bb >= 0; --bb) {
        const int b0 = bb * 16;
        if (w < NSUB) {
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            const double* iu = di + bb * 512 + 256;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int kr = kk * 4 + (lane >> 4);
                acc = mfma4(iu[(lane & 15) * 16 + kr], xs[(b0 + kr) * PX + w * 16 + (lane & 15)], acc);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int v = 0; v < 4; ++v) xs[(b0 + (lane >> 4) + 4 * v) * PX + w * 16 + (lane & 15)] = acc[v];
        }
        __syncthreads();
        for (int job = w; job < bb * NSUB; job += 4) {
            const int st = job / NSUB, sub = job - st * NSUB;
            const int row0 = st * 16, col = sub * 16 + (lane & 15);
            v4d acc;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = xs[(row0 + (lane >> 4) + 4 * v) * PX + col];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int kr = kk * 4 + (lane >> 4);
                const int grow = row0 + (lane & 15), gk = b0 + kr;
                const double av = (gk < M) ? -lu[(size_t)grow * M + gk] : 0.0;
                acc = mfma4(av, xs[(b0 + kr) * PX + col], acc);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) xs[(row0 + (lane >> 4) + 4 * v) * PX + col] = acc[v];
        }
        __syncthreads();
    }
    for (int idx = tid; idx < M * SW; idx += 256) {
        const int rr = idx / SW, c = idx - rr * SW, col = c0 + c;
        if (valid(col)) X[(size_t)rr * ld + col] = xs[rr * PX + c];
    }
}

// Factor mode: RHS = W_i = [C_i | -B_i Y_{i-1}] of chunk blockIdx.y at step t.
// Solve mode: RHS = X_i (R columns).
template <int SW, bool SOLVE>
__global__ __launch_bounds__(256) void k_getrs(const KArgs ka) {
    extern __shared__ double xs[];
    const Level& L = ka.L;
    const int k = blockIdx.y, t = ka.step, M = L.M;
    const int r = chunk_first(L, k), e = chunk_last(L, k);
    if (t > e - r) return;
    const int i = r + t;
    const int c0 = blockIdx.x * SW;
    const int nblk = (M + 15) / 16;
    const double* lu = L.LU + (size_t)i * M * M;
    const double* di = L.DI + (size_t)i * nblk * 512;
    const int* perm = L.perm + (size_t)i * M;
    if (SOLVE) {
        if (c0 >= ka.R) return;
        getrs_slab<SW>(lu, di, perm, ka.X + (size_t)i * M * ka.R, ka.R, M, c0, ka.R, 0, ka.R, 0, 0, xs);
    } else {
        const int e_lo = 0, e_hi = (i != L.N - 1) ? M : 0;
        const int y_lo = M, y_hi = (k > 0) ? 2 * M : M;
        const int c_end = c0 + SW;
        const bool any = (c0 < e_hi && c_end > e_lo) || (c0 < y_hi && c_end > y_lo);
        if (!any) return;
        getrs_slab<SW>(lu, di, perm, L.W + (size_t)i * M * M * 2, 2 * M, M, c0, 2 * M, e_lo, e_hi, y_lo, y_hi, xs);
    }
}

// ------------------------------------------------------------------ small utility kernels

__global__ void k_init_status(unsigned long long* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *st = ~0ULL;
}

// sep table of a level: written from kernel arguments (no host-to-device copy)
__global__ void k_write_ints(int* dst, int count, IntChunk vals) {
    const int t = threadIdx.x;
    if (t < count) dst[t] = vals.v[t];
}

// ------------------------------------------------------------------ residual
//
// r = F - (B X_{i-1} + A X_i + C X_{i+1}); per column sum of squares of r
// and of F.  One workgroup per block row writes its partial sums (no
// atomics: the reduction order is fixed); a second kernel sums them.
__global__ __launch_bounds__(256) void k_residual_rows(int N, int M, int R, const double* __restrict__ A,
                                                      const double* __restrict__ B, const double* __restrict__ C,
                                                      const double* __restrict__ X, const double* __restrict__ F,
                                                      double* __restrict__ part) {
    const int i = blockIdx.x, c = blockIdx.y;
    const size_t MM = (size_t)M * M, MR = (size_t)M * R;
    __shared__ double sr[256], sf[256];
    double accr = 0.0, accf = 0.0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int row = w; row < M; row += 4) {
        double s = 0.0;
        for (int kk = lane; kk < M; kk += 64) {
            s += A[i * MM + (size_t)row * M + kk] * X[i * MR + (size_t)kk * R + c];
            if (i > 0) s += B[i * MM + (size_t)row * M + kk] * X[(i - 1) * MR + (size_t)kk * R + c];
            if (i < N - 1) s += C[i * MM + (size_t)row * M + kk] * X[(i + 1) * MR + (size_t)kk * R + c];
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) {
            const double f = F[i * MR + (size_t)row * R + c];
            const double rv = f - s;
            accr += rv * rv;
            accf += f * f;
        }
    }
    sr[threadIdx.x] = accr;
    sf[threadIdx.x] = accf;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < 4; ++q) { a += sr[q * 64]; b += sf[q * 64]; }
        part[((size_t)c * N + i) * 2 + 0] = a;
        part[((size_t)c * N + i) * 2 + 1] = b;
    }
}

__global__ __launch_bounds__(256) void k_residual_final(int N, int R, const double* __restrict__ part,
                                                       double* __restrict__ out) {
    const int c = blockIdx.x;
    __shared__ double sr[256], sf[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < N; i += 256) {
        a += part[((size_t)c * N + i) * 2 + 0];
        b += part[((size_t)c * N + i) * 2 + 1];
    }
    sr[threadIdx.x] = a;
    sf[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (threadIdx.x < s) { sr[threadIdx.x] += sr[threadIdx.x + s]; sf[threadIdx.x] += sf[threadIdx.x + s]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sf[0] > 0.0 ? sqrt(sr[0]) / sqrt(sf[0]) : sqrt(sr[0]);
}

// ------------------------------------------------------------------ launchers

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

template <int MODE, int NPARTS>
static hipError_t launch_gemm(const KArgs& ka, int batch, int m, int n, hipStream_t s) {
    const int tm = cdiv(m, TB), tn = cdiv(n, TB);
    dim3 grid(tm * tn * NPARTS, batch);
    hipLaunchKernelGGL((k_gemm<MODE, NPARTS>), grid, dim3(256), 0, s, ka, tm, tn);
    return hipGetLastError();
}

hipError_t launch_fwd_gemm(const KArgs& ka, hipStream_t s) { return launch_gemm<GM_FWD, 2>(ka, ka.L.P, ka.L.M, ka.L.M, s); }
hipError_t launch_bwd_gemm(const KArgs& ka, hipStream_t s) { return launch_gemm<GM_BWD, 2>(ka, ka.L.P, ka.L.M, ka.L.M, s); }
hipError_t launch_couple(const KArgs& ka, hipStream_t s) { return launch_gemm<GM_COUPLE, 3>(ka, ka.L.P - 1, ka.L.M, ka.L.M, s); }
hipError_t launch_rhs_fwd(const KArgs& ka, hipStream_t s) { return launch_gemm<GM_RHS_FWD, 1>(ka, ka.L.P, ka.L.M, ka.R, s); }
hipError_t launch_rhs_bwd(const KArgs& ka, hipStream_t s) { return launch_gemm<GM_RHS_BWD, 1>(ka, ka.L.P, ka.L.M, ka.R, s); }
hipError_t launch_couple_rhs(const KArgs& ka, hipStream_t s) { return launch_gemm<GM_COUPLE_RHS, 1>(ka, ka.L.P - 1, ka.L.M, ka.R, s); }
hipError_t launch_recover(const KArgs& ka, hipStream_t s) { return launch_gemm<GM_RECOVER, 1>(ka, ka.L.N, ka.L.M, ka.R, s); }

size_t getrf_lds_bytes(int M) {
    return sizeof(double) * ((size_t)NB * (M + 1) + (size_t)NB * M + 4) + sizeof(int) * (4 + NB + M);
}

hipError_t launch_getrf(const KArgs& ka, hipStream_t s) {
    const size_t lds = getrf_lds_bytes(ka.L.M);
    hipLaunchKernelGGL(k_getrf, dim3(ka.L.P), dim3(256), lds, s, ka);
    return hipGetLastError();
}

static int slab_width(int M) { return M <= 256 ? 32 : 16; }

size_t getrs_lds_bytes(int M) {
    const int sw = slab_width(M);
    return sizeof(double) * (size_t)cdiv(M, 16) * 16 * (sw + 2);
}

hipError_t launch_getrs(const KArgs& ka, bool solve, hipStream_t s) {
    const int M = ka.L.M, sw = slab_width(M);
    const int ncols = solve ? ka.R : 2 * M;
    dim3 grid(cdiv(ncols, sw), ka.L.P);
    const size_t lds = getrs_lds_bytes(M);
    if (sw == 32) {
        if (solve) hipLaunchKernelGGL((k_getrs<32, true>), grid, dim3(256), lds, s, ka);
        else hipLaunchKernelGGL((k_getrs<32, false>), grid, dim3(256), lds, s, ka);
    } else {
        if (solve) hipLaunchKernelGGL((k_getrs<16, true>), grid, dim3(256), lds, s, ka);
        else hipLaunchKernelGGL((k_getrs<16, false>), grid, dim3(256), lds, s, ka);
    }
    return hipGetLastError();
}

hipError_t launch_init_status(unsigned long long* st, hipStream_t s) {
    hipLaunchKernelGGL(k_init_status, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_write_ints(int* dst, const int* host_vals, int count, hipStream_t s) {
    for (int off = 0; off < count; off += IntChunk::CAP) {
        IntChunk c;
        const int n = count - off < IntChunk::CAP ? count - off : IntChunk::CAP;
        for (int q = 0; q < n; ++q) c.v[q] = host_vals[off + q];
        hipLaunchKernelGGL(k_write_ints, dim3(1), dim3(IntChunk::CAP), 0, s, dst + off, n, c);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_residual(int N, int M, int R, const double* A, const double* B, const double* C, const double* X,
                           const double* F, double* out, double* work, hipStream_t s) {
    hipLaunchKernelGGL(k_residual_rows, dim3(N, R), dim3(256), 0, s, N, M, R, A, B, C, X, F, work);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_residual_final, dim3(R), dim3(256), 0, s, N, R, work, out);
    return hipGetLastError();
}

}  // namespace btd

namespace btd {

// Kernels with more than 64 KiB of dynamic LDS must opt in (gfx950 has
// 160 KiB per CU).
hipError_t configure_kernels() {
    const int lds_max = 160 * 1024;
    hipError_t err;
    err = hipFuncSetAttribute((const void*)k_getrf, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (err != hipSuccess) return err;
    err = hipFuncSetAttribute((const void*)k_getrs<32, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (err != hipSuccess) return err;
    err = hipFuncSetAttribute((const void*)k_getrs<32, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (err != hipSuccess) return err;
    err = hipFuncSetAttribute((const void*)k_getrs<16, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (err != hipSuccess) return err;
    return hipFuncSetAttribute((const void*)k_getrs<16, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
}

}  // namespace btd
