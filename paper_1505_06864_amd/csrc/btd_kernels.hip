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

// Output layout of v_mfma_f32_16x16x4f32: 1 when register v of lane l holds
// tile row 4 (l >> 4) + v, 0 when it holds row (l >> 4) + 4 v like the FP64
// instruction.
#ifndef MFMA_F32_ROWS_BY_LANE_GROUP
#define MFMA_F32_ROWS_BY_LANE_GROUP 1
#endif

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

namespace btd {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int chunk_first(const Level& L, int k) { return L.sep[k] + 1; }
__device__ __forceinline__ int chunk_last(const Level& L, int k) { return L.sep[k + 1] - 1; }

__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// FP32 products with FP32 accumulation (the reduced-precision factor).
__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Accumulator of a 16x16 MFMA tile for a product type, and the tile row that
// register v of lane l holds (its column is l & 15).
template <class CT> struct Acc4;
template <> struct Acc4<double> { typedef v4d type; };
template <> struct Acc4<float> { typedef v4f type; };
template <class CT>
__device__ __forceinline__ int mfma_row(int lane, int v) {
    return MFMA_F32_ROWS_BY_LANE_GROUP && sizeof(CT) == 4 ? 4 * (lane >> 4) + v : (lane >> 4) + 4 * v;
}


// Cross-lane helpers.  DPP row permutations reduce within each 16-lane row
// at VALU cost; readlane combines the four rows.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Maximum of an unsigned 32-bit value over the 64 lanes, uniform result:
// one DPP-modified v_max_u32 per stage.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xa, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xc, 0xf, false));
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Sum over the 64 lanes with DPP row operations and four readlanes (the
// same association for every call, so results are deterministic).
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Workgroup copy of n elements with UNR loads in flight per thread before
// the matching stores (a plain strided loop waits for every load).
template <int UNR, class LD, class ST>
__device__ __forceinline__ void copy_batched(int n, LD load, ST store) {
    for (int base = threadIdx.x; base < n; base += 256 * UNR) {
        double v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int idx = base + u * 256;
            v[u] = idx < n ? load(idx) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const int idx = base + u * 256;
            if (idx < n) store(idx, v[u]);
        }
    }
}

#ifdef BTD_PHASE_TIMING
__device__ unsigned long long g_phase[16];
#define PHASE_MARK(var) const unsigned long long var = wall_clock64()
#define PHASE_ADD(slot, a, b) if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) atomicAdd(&g_phase[slot], (b) - (a))
#define PHASE_ADD_W1(slot, a, b) if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 64) atomicAdd(&g_phase[slot], (b) - (a))
#define PHASE_ADD_T(slot, a, b, th) if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == (th)) atomicAdd(&g_phase[slot], (b) - (a))
#else
#define PHASE_MARK(var)
#define PHASE_ADD(slot, a, b)
#define PHASE_ADD_W1(slot, a, b)
#define PHASE_ADD_T(slot, a, b, th)
#endif

// XCD-aware workgroup order.  Workgroups are dispatched round-robin over
// the 8 XCDs (each with its own L2), so dispatch id d runs on XCD d mod 8.
// The logical id returned here makes runs of consecutive logical ids share
// one XCD; a kernel that gives the workgroups of one chunk consecutive
// logical ids keeps that chunk's blocks in one L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_logical_id(int d, int G) {
    const int per = G / NXCD;
    if (d >= per * NXCD) return d;
    return (d % NXCD) * per + d / NXCD;
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
        // chunk c0+b, step t: D_i = A_i - B_i E_{i-1} into the chunk's working copy
        // (part 0, plus C_i -> W_i[:, :M]);
        // Y_i = -B_i Y_{i-1} (part 1, chunks with a left spike).
        const int k = ka.c0 + b, t = ka.step;
        const int r = chunk_first(L, k), e = chunk_last(L, k);
        if (t > e - r) return false;
        const int i = r + t;
        if (part == 0) {
            j.Out = L.Dw + k * MM; j.ldo = M;
            j.Cin = L.A + i * MM; j.ldc = M;
            if (t > 0) { j.A1 = L.B + i * MM; j.lda1 = M; j.B1 = L.W + (i - 1) * MM * 2; j.ldb1 = M2; j.k1 = M; }
            // C_i -> W_i[:, :M] only for the workgroup slab solve (M > 256); the
            // wave-slab solve reads C_i itself
            if (i != L.N - 1 && M > 256) { j.CopyIn = L.C + i * MM; j.ldci = M; j.CopyOut = L.W + i * MM * 2; j.ldco = M2; }
            return true;
        }
        if (k == 0) return false;
        j.Out = L.W + i * MM * 2 + M; j.ldo = M2;
        if (t == 0) { j.Cin = L.B + i * MM; j.ldc = M; }
        else { j.A1 = L.B + i * MM; j.lda1 = M; j.B1 = L.W + (i - 1) * MM * 2 + M; j.ldb1 = M2; j.k1 = M; }
        return true;
    } else if (MODE == GM_BWD) {
        // chunk c0+b, backward step s (row i = e - s): Z_L (part 0, k > 0), Z_R (part 1, k < P-1)
        const int k = ka.c0 + b, s = ka.step;
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
    } else if (MODE == GM_COUPLE_RHS) {
        const int jj = b, q = L.sep[jj + 1], R = ka.R;
        const size_t MR = (size_t)M * R;
        j.n = R;
        j.Out = ka.Fc + jj * MR; j.ldo = R;
        j.Cin = ka.F + q * MR; j.ldc = R;
        j.A1 = L.B + q * MM; j.lda1 = M; j.B1 = ka.X + (q - 1) * MR; j.ldb1 = R; j.k1 = M;
        j.A2 = L.C + q * MM; j.lda2 = M; j.B2 = ka.X + (q + 1) * MR; j.ldb2 = R; j.k2 = M;
        return true;
    } else if (MODE == GM_RHS_FWD) {
        // right-hand-side sweep, chunk c0+b, step t: X_i = F_i - B_i X_{i-1}
        // (X_{i-1} already solved), before the LU solve of row i
        const int k = ka.c0 + b, t = ka.step, R = ka.R;
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
        // right-hand-side sweep, chunk c0+b, backward step s (row i = e-1-s):
        // X_i -= E_i X_{i+1}
        const int k = ka.c0 + b, s = ka.step, R = ka.R;
        const int r = chunk_first(L, k), e = chunk_last(L, k);
        if (s > e - r - 1) return false;
        const int i = e - 1 - s;
        const size_t MR = (size_t)M * R;
        j.n = R;
        j.Out = ka.X + i * MR; j.ldo = R;
        j.Cin = ka.X + i * MR; j.ldc = R;
        j.A1 = L.W + i * MM * 2; j.lda1 = M2; j.B1 = ka.X + (i + 1) * MR; j.ldb1 = R; j.k1 = M;
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
// LDS: two buffers of As[16][64+AP] (k-major, transposed) and Bs[16][64+BP];
// the next K step is loaded (32-byte pieces when the rows are 32-byte
// aligned) while the current one is multiplied, one barrier per K step.
// AP = 3: the transposed stores of As (lanes 4 k-rows apart writing the
// same tile row) then fall in different LDS banks (with a pad of 4 they
// collided four ways).
constexpr int TB = 64, KB = 16, AP = 3, BP = 4;
constexpr int ASZ = KB * (TB + AP), BSZ = KB * (TB + BP);

template <bool FULL>
__device__ __forceinline__ void load_tiles(const double* __restrict__ A, int lda, const double* __restrict__ Bm,
                                           int ldb, int row0, int col0, int k0, int m, int n, int K, double ra[4],
                                           double rb[4]) {
    const int tid = threadIdx.x;
    {
        const int rr = tid >> 2, kq = (tid & 3) * 4;
        const int gr = row0 + rr, gk = k0 + kq;
        if (FULL || (gr < m && gk + 3 < K && (lda & 3) == 0)) {
            const double4 x = *(const double4*)(A + (size_t)gr * lda + gk);
            ra[0] = x.x; ra[1] = x.y; ra[2] = x.z; ra[3] = x.w;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) ra[q] = (gr < m && gk + q < K) ? A[(size_t)gr * lda + gk + q] : 0.0;
        }
    }
    {
        const int kk = tid >> 4, cq = (tid & 15) * 4;
        const int gk = k0 + kk, gc = col0 + cq;
        if (FULL || (gk < K && gc + 3 < n && (ldb & 3) == 0)) {
            const double4 x = *(const double4*)(Bm + (size_t)gk * ldb + gc);
            rb[0] = x.x; rb[1] = x.y; rb[2] = x.z; rb[3] = x.w;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) rb[q] = (gk < K && gc + q < n) ? Bm[(size_t)gk * ldb + gc + q] : 0.0;
        }
    }
}

// The tiles go to LDS in the product type CT (FP64 values rounded to FP32
// for the reduced-precision factor).
template <class CT>
__device__ __forceinline__ void store_tiles(CT* As, CT* Bs, const double ra[4], const double rb[4]) {
    const int tid = threadIdx.x;
    {
        const int rr = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) As[(kq + q) * (TB + AP) + rr] = (CT)ra[q];
    }
    {
        const int kk = tid >> 4, cq = (tid & 15) * 4;
        if constexpr (sizeof(CT) == 8) {
            *(double4*)(Bs + kk * (TB + BP) + cq) = make_double4(rb[0], rb[1], rb[2], rb[3]);
        } else {
            *(float4*)(Bs + kk * (TB + BP) + cq) = make_float4((float)rb[0], (float)rb[1], (float)rb[2], (float)rb[3]);
        }
    }
}

template <class CT>
__device__ __forceinline__ void tile_mma(const CT* as, const CT* bs, int lane, int wr, int wc,
                                         typename Acc4<CT>::type acc[2][2]) {
#pragma unroll
    for (int kk = 0; kk < KB / 4; ++kk) {
        const int krow = kk * 4 + (lane >> 4);
        CT a0 = as[krow * (TB + AP) + wr + (lane & 15)];
        CT a1 = as[krow * (TB + AP) + wr + 16 + (lane & 15)];
        CT b0 = bs[krow * (TB + BP) + wc + (lane & 15)];
        CT b1 = bs[krow * (TB + BP) + wc + 16 + (lane & 15)];
        acc[0][0] = mfma4(a0, b0, acc[0][0]);
        acc[0][1] = mfma4(a0, b1, acc[0][1]);
        acc[1][0] = mfma4(a1, b0, acc[1][0]);
        acc[1][1] = mfma4(a1, b1, acc[1][1]);
    }
}

// The global loads run two K steps ahead of the products: while step s is
// multiplied from one LDS buffer, step s+1 (loaded during step s-1) goes
// from registers into the other buffer and step s+2 is in flight in a
// second register set, so a load has two steps of products to arrive.
// FULL: the tile lies inside the matrix, K is a multiple of two K steps and
// the rows are 32-byte aligned; every load is then unconditional (the last
// two steps load the final K step again, unused), which keeps the loop free
// of branches, so the loads of step s+2 stay in flight while step s+1 is
// stored.
template <bool FULL, class CT>
__device__ void tile_accumulate_k(const double* __restrict__ A, int lda, const double* __restrict__ Bm, int ldb,
                                  int K, int row0, int col0, int m, int n, typename Acc4<CT>::type acc[2][2], CT* As,
                                  CT* Bs) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    double ra0[4], rb0[4], ra1[4], rb1[4];
    const int nk = (K + KB - 1) / KB;
    load_tiles<FULL>(A, lda, Bm, ldb, row0, col0, 0, m, n, K, ra0, rb0);
    if (FULL || nk > 1) load_tiles<FULL>(A, lda, Bm, ldb, row0, col0, KB, m, n, K, ra1, rb1);
    __syncthreads();   // the buffers may still be read by a previous accumulation
    store_tiles(As, Bs, ra0, rb0);
    __syncthreads();
    if constexpr (FULL) {
        for (int s = 0; s < nk; s += 2) {
            load_tiles<true>(A, lda, Bm, ldb, row0, col0, min(s + 2, nk - 1) * KB, m, n, K, ra0, rb0);
            tile_mma(As, Bs, lane, wr, wc, acc);
            store_tiles(As + ASZ, Bs + BSZ, ra1, rb1);
            __syncthreads();
            load_tiles<true>(A, lda, Bm, ldb, row0, col0, min(s + 3, nk - 1) * KB, m, n, K, ra1, rb1);
            tile_mma(As + ASZ, Bs + BSZ, lane, wr, wc, acc);
            store_tiles(As, Bs, ra0, rb0);
            __syncthreads();
        }
    } else {
        for (int s = 0; s < nk; s += 2) {
            // step s from buffer 0; step s+1 in ra1/rb1; ra0/rb0 free
            if (s + 2 < nk) load_tiles<false>(A, lda, Bm, ldb, row0, col0, (s + 2) * KB, m, n, K, ra0, rb0);
            tile_mma(As, Bs, lane, wr, wc, acc);
            if (s + 1 < nk) store_tiles(As + ASZ, Bs + BSZ, ra1, rb1);
            __syncthreads();
            if (s + 1 >= nk) break;
            // step s+1 from buffer 1; step s+2 in ra0/rb0; ra1/rb1 free
            if (s + 3 < nk) load_tiles<false>(A, lda, Bm, ldb, row0, col0, (s + 3) * KB, m, n, K, ra1, rb1);
            tile_mma(As + ASZ, Bs + BSZ, lane, wr, wc, acc);
            if (s + 2 < nk) store_tiles(As, Bs, ra0, rb0);
            __syncthreads();
        }
    }
}

template <class CT>
__device__ void tile_accumulate(const double* __restrict__ A, int lda, const double* __restrict__ Bm, int ldb,
                                int K, int row0, int col0, int m, int n, typename Acc4<CT>::type acc[2][2], CT* As,
                                CT* Bs) {
    if (K <= 0) return;
    const bool full = row0 + TB <= m && col0 + TB <= n && K % (2 * KB) == 0 && (lda & 3) == 0 &&
                      (ldb & 3) == 0 && ((uintptr_t)A & 31) == 0 && ((uintptr_t)Bm & 31) == 0;
    if (full) tile_accumulate_k<true, CT>(A, lda, Bm, ldb, K, row0, col0, m, n, acc, As, Bs);
    else tile_accumulate_k<false, CT>(A, lda, Bm, ldb, K, row0, col0, m, n, acc, As, Bs);
}

// At most 128 VGPRs (four waves per SIMD, as many as the LDS admits) except
// for the coupling right-hand sides, whose job set-up needs more.
// CT: product type (double; float = FP32 products with FP32 accumulation,
// added to the FP64 Cin in FP64).
template <int MODE, int NPARTS, class CT = double>
__global__ __launch_bounds__(256, MODE == GM_COUPLE_RHS ? 3 : 4) void k_gemm(const KArgs ka, int tiles_m, int tiles_n) {
    __shared__ CT As[2 * ASZ];
    __shared__ CT Bs[2 * BSZ];
    const int per_item = tiles_m * tiles_n * NPARTS;
    const int lid = xcd_logical_id(blockIdx.x, gridDim.x);
    const int b = lid / per_item;
    int bx = lid % per_item;
    const int tn = bx % tiles_n; bx /= tiles_n;
    const int tm = bx % tiles_m; bx /= tiles_m;
    const int part = bx;
    Job j;
    if (!make_job<MODE>(ka, b, part, j)) return;
    const int row0 = tm * TB, col0 = tn * TB;
    if (row0 >= j.m || col0 >= j.n) return;
    typename Acc4<CT>::type acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = (typename Acc4<CT>::type){0, 0, 0, 0};
    tile_accumulate<CT>(j.A1, j.lda1, j.B1, j.ldb1, j.k1, row0, col0, j.m, j.n, acc, As, Bs);
    tile_accumulate<CT>(j.A2, j.lda2, j.B2, j.ldb2, j.k2, row0, col0, j.m, j.n, acc, As, Bs);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = row0 + (w >> 1) * 32, wc = col0 + (w & 1) * 32;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int col = wc + 16 * c + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wr + 16 * a + mfma_row<CT>(lane, v);
                if (row < j.m && col < j.n) {
                    double base = j.Cin ? j.Cin[(size_t)row * j.ldc + col] : 0.0;
                    j.Out[(size_t)row * j.ldo + col] = base + j.alpha * (double)acc[a][c][v];
                    if (j.CopyOut) j.CopyOut[(size_t)row * j.ldco + col] = j.CopyIn[(size_t)row * j.ldci + col];
                }
            }
        }
}

// ------------------------------------------------------------------ LU
//
// LU with partial pivoting of every D_i factored at this step, one
// workgroup of NT threads per block (NT >= M), right-looking with panels of
// NB columns, on the chunk's working copy of D_i.  Rows never move in the
// working copy: thread t owns row t.  As soon as a panel's NB pivot rows are
// known and eliminated they are final and are written to the factor array
// in pivot order (their multipliers from the working copy, the panel part
// and U12 from LDS), so the factors come out in pivot order with
// perm[q] = the row of D_i chosen as q-th pivot.
//   panel   every thread keeps the NB panel values of its row in registers.
//           Per column: each wave finds its largest |value| among the rows
//           not chosen yet (DPP reduction) and publishes value, row and the
//           rest of that row to a double-buffered LDS slot; after one
//           barrier every thread takes the overall maximum (lowest row on
//           ties; a non-finite value always wins so that it is reported)
//           and eliminates with the pivot row read back from the slot.
//   U12     inv(L11) of the panel's unit lower triangle, then
//           U12 = inv(L11) A12 on MFMA for the pivot rows right of the panel.
//   update  A22 -= L21 U12 on MFMA over the rows not chosen yet, which are
//           listed contiguously, in 32 x 32 tiles spread over the waves.
constexpr int DB = 32;                 // diagonal block of the triangular solves
constexpr int DI_STRIDE = 2 * DB * DB; // doubles per diagonal block (L inverse, then U inverse)

__device__ __forceinline__ void wave_lds_sync() { __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

struct LuLds {
    int LP, UP, TP;   // pitches (doubles) of the multiplier rows, U12 rows, inv(L11) rows
    size_t lb, ub, tb, cval, crow, cidx, piv, list, wcnt, total;
};

// LP = NB + 2 and UP = 16 (mod 32) keep the MFMA operand reads of one
// 32-lane half free of bank conflicts for consecutive rows.
__host__ __device__ inline LuLds lu_lds_layout(int M, int NT, int NB) {
    LuLds l;
    const int NW = NT / 64;
    l.LP = NB + 2;
    l.TP = NB + 2;
    const int w2 = M > NB ? M - NB : 1;
    l.UP = ((w2 + 31) / 32) * 32 + 16;
    size_t off = 0;
    l.lb = off; off += sizeof(double) * (size_t)NT * l.LP;
    l.ub = off; off += sizeof(double) * (size_t)NB * l.UP;
    l.tb = off; off += sizeof(double) * (size_t)NB * l.TP;
    l.cval = off; off += sizeof(double) * 2 * NW * 4;
    l.crow = off; off += sizeof(double) * 2 * NW * (size_t)NB;
    l.cidx = off; off += sizeof(int) * 2 * NW;
    l.piv = off; off += sizeof(int) * NB;
    l.list = off; off += sizeof(int) * (size_t)NT;
    l.wcnt = off; off += sizeof(int) * (NW + 1);
    l.total = (off + 15) & ~(size_t)15;
    return l;
}

// The column steps of one panel.  Thread t holds the panel row t in v.
// Pivot search per column: key = bits(|value|) + 1 for rows not chosen yet
// (non-finite values count as +inf so that they win and are reported),
// 0 otherwise; its high word is reduced with 32-bit DPP maxima, and only
// when several lanes share the maximal high word the low word decides among
// them (lowest lane on exact ties).  The wave's winner publishes its key,
// the reciprocal of its value (two Newton steps from v_rcp_f64), its row and
// its value in the next column to a 32-byte slot, and the rest of its row to
// crow; after the barrier every thread picks the largest key (lowest wave on
// ties) without a dependent LDS read and eliminates.
template <int NT, int NB, bool FULL>
__device__ __forceinline__ void lu_panel_steps(double (&v)[NB], bool& act, int& mypos, int& fail_code, int& fail_col,
                                               int j0, int nb, int row, int lane, int w, double* cslot, double* crow) {
    constexpr int NW = NT / 64;
    constexpr unsigned long long KINF = 0x7FF0000000000001ull;   // key of a non-finite value
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) {
        if (jj < nb) {
            PHASE_MARK(t_s0);
            const int par = jj & 1;
            const double vj = v[jj];
            const unsigned long long bits =
                isfinite(vj) ? (unsigned long long)__double_as_longlong(fabs(vj)) + 1ull : KINF;
            const unsigned long long key = act ? bits : 0ull;
            double r = __builtin_amdgcn_rcp(vj);
            r = fma(r, fma(-vj, r, 1.0), r);
            r = fma(r, fma(-vj, r, 1.0), r);
            const unsigned hi = (unsigned)(key >> 32);
            const unsigned mhi = wave_max_u32(hi);
            unsigned long long tied = __ballot(hi == mhi);
            if (__popcll(tied) > 1) {
                const unsigned lo = hi == mhi ? (unsigned)key : 0u;
                const unsigned mlo = wave_max_u32(lo);
                tied = __ballot(hi == mhi && lo == mlo);
            }
            const int wl = __ffsll((unsigned long long)tied) - 1;
            if (lane == wl) {
                double* sl = cslot + (par * NW + w) * 4;
                sl[0] = __longlong_as_double((long long)key);
                sl[1] = r;
                sl[2] = (double)row;
                if (jj + 1 < NB) sl[3] = v[jj + 1];
                double* cr = crow + (size_t)(par * NW + w) * NB;
#pragma unroll
                for (int c = jj + 2; c < NB; ++c) cr[c] = v[c];
            }
            PHASE_MARK(t_s1);
            __syncthreads();
            PHASE_MARK(t_s2);
            PHASE_ADD(5, t_s0, t_s1);
            PHASE_ADD(6, t_s1, t_s2);
            // the four keys first (independent reads), then everything of the
            // winning wave in one round of reads
            const unsigned long long* skey = (const unsigned long long*)cslot;
            unsigned long long kq[NW];
#pragma unroll
            for (int q = 0; q < NW; ++q) kq[q] = skey[(par * NW + q) * 4];
            unsigned long long bk = kq[0];
            int bw = 0;
#pragma unroll
            for (int q = 1; q < NW; ++q) {
                const bool tk = kq[q] > bk;
                bk = tk ? kq[q] : bk;
                bw = tk ? q : bw;
            }
            const double* sl = cslot + (par * NW + bw) * 4;
            const double rcp = sl[1], prw = sl[2], p1 = sl[3];
            const bool bad = bk == 1ull || bk == KINF;   // |pivot| zero or non-finite
            if (bad && fail_code == 0) {
                fail_code = bk == 1ull ? BTD_ERR_SINGULAR_ : BTD_ERR_NONFINITE_;
                fail_col = j0 + jj;
            }
            const double rp = bad ? 0.0 : rcp;
            const bool me = row == (int)prw;
            mypos = me ? j0 + jj : mypos;
            act = act && !me;
            const double l = act ? vj * rp : 0.0;
            v[jj] = act ? l : vj;
            if (jj + 1 < NB) v[jj + 1] = fma(-l, p1, v[jj + 1]);
            const double* pr = crow + (size_t)(par * NW + bw) * NB;
#pragma unroll
            for (int c = jj + 2; c < NB; ++c) v[c] = fma(-l, pr[c], v[c]);
            PHASE_MARK(t_s3);
            PHASE_ADD(7, t_s2, t_s3);
        }
    }
}

template <int NT, int NB>
__global__ __launch_bounds__(NT) void k_getrf(const KArgs ka) {
    constexpr int NW = NT / 64;
    constexpr int KS = NB / 4;   // MFMA k-steps per panel
    const Level& L = ka.L;
    const int kch = ka.c0 + blockIdx.x, t = ka.step;
    const int r0 = chunk_first(L, kch), e = chunk_last(L, kch);
    if (t > e - r0) return;
    const int i = r0 + t;
    const int M = L.M;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4;
    double* a = L.Dw + (size_t)kch * M * M;      // working copy, rows in place
    double* out = L.LU + (size_t)i * M * M;      // factors, rows in pivot order
    extern __shared__ double sm_raw[];
    char* smc = (char*)sm_raw;
    const LuLds lay = lu_lds_layout(M, NT, NB);
    const int LP = lay.LP, UP = lay.UP, TP = lay.TP;
    double* Lb = (double*)(smc + lay.lb);
    double* Ub = (double*)(smc + lay.ub);
    double* Tb = (double*)(smc + lay.tb);
    double* cslot = (double*)(smc + lay.cval);   // [2][NW][4]: |value|, reciprocal, row
    double* crow = (double*)(smc + lay.crow);
    int* piv = (int*)(smc + lay.piv);
    int* list = (int*)(smc + lay.list);
    int* wcnt = (int*)(smc + lay.wcnt);

    const int row = tid;
    bool act = row < M;
    int mypos = -1;
    int fail_code = 0, fail_col = -1;   // identical in every thread
    const int npan = (M + NB - 1) / NB;
    double vn[NB];   // the next panel's values of this thread's row
#pragma unroll
    for (int c = 0; c < NB; ++c) vn[c] = (act && c < M) ? a[(size_t)row * M + c] : 0.0;
    for (int p = 0; p < npan; ++p) {
        const int j0 = p * NB, nb = min(NB, M - j0);
        PHASE_MARK(t_p0);
        double v[NB];
        const bool act0 = act;
#pragma unroll
        for (int c = 0; c < NB; ++c) v[c] = vn[c];

        // ---------------- panel
        if (nb == NB) lu_panel_steps<NT, NB, true>(v, act, mypos, fail_code, fail_col, j0, nb, row, lane, w, cslot, crow);
        else lu_panel_steps<NT, NB, false>(v, act, mypos, fail_code, fail_col, j0, nb, row, lane, w, cslot, crow);
        PHASE_MARK(t_p1);
        PHASE_ADD(0, t_p0, t_p1);
        // the panel, factored, to the multiplier rows (every row active at the
        // panel's start) and, for the rows not chosen yet, to the working copy;
        // the pivot order of the panel; the rows not chosen yet
        if (act0) {
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                Lb[row * LP + c] = v[c];
                if (act && c < nb) a[(size_t)row * M + j0 + c] = v[c];   // read back when the row is chosen
            }
        }
        if (mypos >= j0 && mypos < j0 + nb) piv[mypos - j0] = row;
        {
            const unsigned long long am = __ballot(act);
            if (lane == 0) wcnt[w] = __popcll(am);
            __syncthreads();
            int base = 0;
#pragma unroll
            for (int q = 0; q < NW; ++q) base += q < w ? wcnt[q] : 0;
            if (act) list[base + __popcll(am & ((1ull << lane) - 1ull))] = row;
        }
        const int w2 = M - j0 - nb;   // columns right of the panel (0 only after the last panel)
        // ---------------- the pivot rows, read once from the working copy: the
        // multipliers left of the panel go to the factors, A12 to Ub
        {
            constexpr int RW = (NB + NW - 1) / NW, CL = NT / 64;
            double val[RW][CL];
#pragma unroll
            for (int q = 0; q < RW; ++q) {
                const int rr = w + q * NW;
                const int pr = rr < nb ? piv[rr] : 0;
#pragma unroll
                for (int u = 0; u < CL; ++u) {
                    const int c = lane + 64 * u;
                    val[q][u] = (rr < nb && c < M && (c < j0 || c >= j0 + nb)) ? a[(size_t)pr * M + c] : 0.0;
                }
            }
#pragma unroll
            for (int q = 0; q < RW; ++q) {
                const int rr = w + q * NW;
                if (rr < nb) {
                    const int pr = piv[rr];
#pragma unroll
                    for (int u = 0; u < CL; ++u) {
                        const int c = lane + 64 * u;
                        if (c < j0) out[(size_t)(j0 + rr) * M + c] = val[q][u];
                        else if (c < j0 + nb) out[(size_t)(j0 + rr) * M + c] = Lb[pr * LP + c - j0];
                        else if (c < M) Ub[rr * UP + c - j0 - nb] = val[q][u];
                    }
                }
            }
        }
        PHASE_MARK(t_p2);
        PHASE_ADD(1, t_p1, t_p2);
        if (w2 <= 0) break;
        __syncthreads();
        // ---------------- inv(L11): two 16 x 16 diagonal blocks by forward
        // substitution (lanes 0..15 the first, 16..31 the second), then the
        // off-diagonal block -inv(L_22) L_21 inv(L_11) on MFMA.
        if (w == 0 && lane < NB) {
            const int half = lane / 16, jc = lane % 16, o = half * 16;
            double x[16];
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) {
                double s = (rr == jc) ? 1.0 : 0.0;
                const double* lr = Lb + piv[o + rr] * LP + o;
#pragma unroll
                for (int c = 0; c < rr; ++c) s = fma(-lr[c], x[c], s);
                x[rr] = rr >= jc ? s : 0.0;
            }
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) Tb[(o + rr) * TP + o + jc] = x[rr];
            if (NB == 32) {
#pragma unroll
                for (int rr = 0; rr < 16; ++rr) Tb[rr * TP + 16 + jc] = 0.0;
            }
        }
        __syncthreads();
        if (NB == 32 && w == 0) {
            // W = L_21 inv(L_11) (16 x 16), then T_21 = -inv(L_22) W
            v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                acc = mfma4(Lb[piv[16 + (lane & 15)] * LP + 4 * kk + g], Tb[(4 * kk + g) * TP + (lane & 15)], acc);
            double* wt = crow;   // 16 x 16 scratch (the candidate slots are free here)
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) wt[(g + 4 * vv) * 16 + (lane & 15)] = acc[vv];
            wave_lds_sync();
            v4d acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                acc2 = mfma4(-Tb[(16 + (lane & 15)) * TP + 16 + 4 * kk + g], wt[(4 * kk + g) * 16 + (lane & 15)], acc2);
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) Tb[(16 + g + 4 * vv) * TP + (lane & 15)] = acc2[vv];
        }
        __syncthreads();
        // ---------------- U12 = inv(L11) A12 in place in Ub, 16-column strips over
        // the waves; the rows of U12 are final and go to the factors too
        for (int cs = w * 16; cs < w2; cs += NW * 16) {
            const int col = cs + (lane & 15);
            double bop[KS];
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) bop[kk] = col < w2 ? Ub[(4 * kk + g) * UP + col] : 0.0;
#pragma unroll
            for (int x = 0; x < NB / 16; ++x) {
                v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < KS; ++kk) acc = mfma4(Tb[(16 * x + (lane & 15)) * TP + 4 * kk + g], bop[kk], acc);
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    const int rr = 16 * x + g + 4 * vv;
                    Ub[rr * UP + col] = acc[vv];
                    if (col < w2) out[(size_t)(j0 + rr) * M + j0 + nb + col] = acc[vv];
                }
            }
        }
        __syncthreads();
        PHASE_MARK(t_p3);
        PHASE_ADD(2, t_p2, t_p3);
        // ---------------- A22 -= L21 U12 over the rows not chosen yet (list) in
        // 32 x 32 tiles: first the next panel's columns, then every thread
        // starts loading its row of the next panel while the other tiles are
        // updated with their loads three tiles ahead.
        const int h2 = w2;
        const int tr_n = (h2 + 31) / 32, tc_n = (w2 + 31) / 32;
        double* a2 = a + j0 + nb;
        auto load_tile = [&](int tr, int tc, v4d (&c)[2][2], int (&crw)[2][4]) {
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    const int idx = tr + 16 * x + g + 4 * vv;
                    crw[x][vv] = idx < h2 ? list[idx] : -1;
                }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    const int col = tc + 16 * y + (lane & 15);
#pragma unroll
                    for (int vv = 0; vv < 4; ++vv)
                        c[x][y][vv] = (crw[x][vv] >= 0 && col < w2) ? a2[(size_t)crw[x][vv] * M + col] : 0.0;
                }
        };
        auto mul_store = [&](int tr, int tc, v4d (&c)[2][2], const int (&crw)[2][4]) {
            int arw[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int idx = tr + 16 * x + (lane & 15);
                arw[x] = idx < h2 ? list[idx] : -1;
            }
#pragma unroll
            for (int kk = 0; kk < KS; ++kk) {
                double av[2], bv[2];
#pragma unroll
                for (int x = 0; x < 2; ++x) av[x] = arw[x] >= 0 ? -Lb[arw[x] * LP + 4 * kk + g] : 0.0;
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    const int col = tc + 16 * y + (lane & 15);
                    bv[y] = col < w2 ? Ub[(4 * kk + g) * UP + col] : 0.0;
                }
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y) c[x][y] = mfma4(av[x], bv[y], c[x][y]);
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    const int col = tc + 16 * y + (lane & 15);
#pragma unroll
                    for (int vv = 0; vv < 4; ++vv)
                        if (crw[x][vv] >= 0 && col < w2) a2[(size_t)crw[x][vv] * M + col] = c[x][y][vv];
                }
        };
        {
            v4d c0[2][2];
            int q0[2][4];
            for (int s = w; s < tr_n; s += NW) {
                load_tile(s * 32, 0, c0, q0);
                mul_store(s * 32, 0, c0, q0);
            }
        }
        __syncthreads();
        PHASE_MARK(t_p4);
        PHASE_ADD(3, t_p3, t_p4);
        {
            const int j1 = j0 + nb, nb1 = min(NB, M - j1);
#pragma unroll
            for (int c = 0; c < NB; ++c) vn[c] = (act && c < nb1) ? a[(size_t)row * M + j1 + c] : 0.0;
        }
        {
            const int tcr = tc_n - 1, nrest = tr_n * tcr;
            v4d b0[2][2], b1[2][2], b2[2][2];
            int q0[2][4], q1[2][4], q2[2][4];
#define LU_T(s) ((s) / tcr) * 32, (1 + (s) % tcr) * 32
            int s = w;
            if constexpr (NW == 4) {
                // three tiles in flight: the current one and two ahead
                if (s < nrest) load_tile(LU_T(s), b0, q0);
                if (s + NW < nrest) load_tile(LU_T(s + NW), b1, q1);
                for (; s < nrest; s += 3 * NW) {
                    if (s + 2 * NW < nrest) load_tile(LU_T(s + 2 * NW), b2, q2);
                    mul_store(LU_T(s), b0, q0);
                    if (s + NW >= nrest) break;
                    if (s + 3 * NW < nrest) load_tile(LU_T(s + 3 * NW), b0, q0);
                    mul_store(LU_T(s + NW), b1, q1);
                    if (s + 2 * NW >= nrest) break;
                    if (s + 4 * NW < nrest) load_tile(LU_T(s + 4 * NW), b1, q1);
                    mul_store(LU_T(s + 2 * NW), b2, q2);
                }
            } else {
                // eight waves: half the registers per wave, one tile ahead
                if (s < nrest) load_tile(LU_T(s), b0, q0);
                for (; s < nrest; s += 2 * NW) {
                    if (s + NW < nrest) load_tile(LU_T(s + NW), b1, q1);
                    mul_store(LU_T(s), b0, q0);
                    if (s + NW >= nrest) break;
                    if (s + 2 * NW < nrest) load_tile(LU_T(s + 2 * NW), b0, q0);
                    mul_store(LU_T(s + NW), b1, q1);
                }
            }
#undef LU_T
        }
        __syncthreads();
        PHASE_MARK(t_p5);
        PHASE_ADD(4, t_p4, t_p5);
    }
    int* perm = L.perm + (size_t)i * M;
    if (mypos >= 0) perm[mypos] = row;
    if (tid == 0 && fail_code != 0) report_status(ka.status, L.level, i, fail_col, fail_code);
}

// ------------------------------------------------------------------ LU, one panel wave
//
// The factorisation of k_getrf (rows fixed in the working copy, factors
// written in pivot order) for M <= 256 with the pivot chain on a single
// wave, so that a column step needs no workgroup synchronisation: wave 0
// holds rows 4l .. 4l+3 of a 16-column panel in lane l (64 registers of
// doubles) and finds each pivot with a lane-local maximum and a DPP maximum;
// the pivot's lane passes the rest of the pivot row through LDS (a 16-value
// slot, written by one lane and read back by all).  Waves 1..7 work one
// panel behind:
// while wave 0 factors panel p they apply panel p-1 to the columns right of
// panel p (U12 = inv(L11) A12 and A22 -= L21 U12 in 16-column slabs on MFMA)
// and copy the finished factor rows; the columns of panel p+1 are kept in
// LDS.  Between panels only the next panel's columns are brought up to date
// (U12 of those 16 columns, then 16 columns of the update on all waves).
// Ties in the pivot search go to the lowest row, as in the other kernels.
constexpr int LW_NB = 16, LW_NT = 512, LW_HW = LW_NT / 64 - 1;   // panel width, threads, helper waves
constexpr int LW_P = LW_NB + 1;                                  // LDS row pitch (doubles)

struct LwLds {
    size_t nx, lb, tb, un, list, piv, prow, total;
};

// nx: the columns of the next two panels, [2][256][LW_P] by row; lb: the
// panel rows (multipliers, pivot rows) of the last two panels, by row;
// tb: inv(L11); un: U12 of the next panel; list: rows not yet chosen, in
// row order, of the last two panels; piv: pivot rows of the last two panels;
// prow: the pivot row of the current column step.
__host__ __device__ constexpr LwLds lw_lds_layout() {
    LwLds l{};
    size_t off = 0;
    l.nx = off; off += sizeof(double) * 2 * 256 * LW_P;
    l.lb = off; off += sizeof(double) * 2 * 256 * LW_P;
    l.tb = off; off += sizeof(double) * LW_NB * LW_P;
    l.un = off; off += sizeof(double) * LW_NB * LW_P;
    l.list = off; off += sizeof(int) * 2 * 256;
    l.piv = off; off += sizeof(int) * 2 * LW_NB;
    l.prow = off; off += sizeof(double) * LW_NB;
    l.total = (off + 15) & ~(size_t)15;
    return l;
}

// The column steps of one panel on one wave; v[r][c] is column j0+c of row
// 4*lane+r, act[r] whether that row is still a candidate.
__device__ __forceinline__ void lw_panel_steps(double (&v)[4][LW_NB], bool (&act)[4], int& fail_code, int& fail_col,
                                               int j0, int nb, int lane, int* piv, double* prow) {
    constexpr int NB = LW_NB;
    constexpr unsigned long long KINF = 0x7FF0000000000001ull;
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) {
        if (jj < nb) {
            // the lane's candidate: largest |value| of its rows, lowest row on ties
            unsigned long long kb = 0ull;
            int rb = 0;
            double vb = 1.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double x = v[r][jj];
                const unsigned long long bits =
                    isfinite(x) ? (unsigned long long)__double_as_longlong(fabs(x)) + 1ull : KINF;
                const unsigned long long key = act[r] ? bits : 0ull;
                const bool tk = key > kb;
                kb = tk ? key : kb;
                rb = tk ? r : rb;
                vb = tk ? x : vb;
            }
            double rc = __builtin_amdgcn_rcp(vb);
            rc = fma(rc, fma(-vb, rc, 1.0), rc);
            rc = fma(rc, fma(-vb, rc, 1.0), rc);
            // the wave's maximum key; its lowest lane holds the lowest row
            const unsigned hi = (unsigned)(kb >> 32);
            const unsigned mhi = wave_max_u32(hi);
            unsigned long long tied = __ballot(hi == mhi);
            if (__popcll(tied) > 1) {
                const unsigned lo = hi == mhi ? (unsigned)kb : 0u;
                const unsigned mlo = wave_max_u32(lo);
                tied = __ballot(hi == mhi && lo == mlo);
            }
            const int wl = __ffsll((unsigned long long)tied) - 1;
            const int rs = __builtin_amdgcn_readlane(rb, wl);
            const unsigned long long bk =
                ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(kb >> 32), wl) << 32) |
                (unsigned)__builtin_amdgcn_readlane((int)kb, wl);
            const bool bad = bk == 1ull || bk == KINF;
            if (bad && fail_code == 0) {
                fail_code = bk == 1ull ? BTD_ERR_SINGULAR_ : BTD_ERR_NONFINITE_;
                fail_col = j0 + jj;
            }
            const double rp = bad ? 0.0 : readlane_d(rc, wl);
            if (lane == 0) piv[jj] = 4 * wl + rs;
            // the rest of the pivot row, through LDS from its lane
            if (rs == 0) {
                if (lane == wl) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) if (c > jj) prow[c] = v[0][c];
                }
                __asm__ volatile("; pivot row in slot 0");
            } else if (rs == 1) {
                if (lane == wl) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) if (c > jj) prow[c] = v[1][c];
                }
                __asm__ volatile("; pivot row in slot 1");
            } else if (rs == 2) {
                if (lane == wl) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) if (c > jj) prow[c] = v[2][c];
                }
                __asm__ volatile("; pivot row in slot 2");
            } else {
                if (lane == wl) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) if (c > jj) prow[c] = v[3][c];
                }
                __asm__ volatile("; pivot row in slot 3");
            }
            wave_lds_sync();
            double pr[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) pr[c] = c > jj ? prow[c] : 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool me = lane == wl && r == rs;
                act[r] = act[r] && !me;
                const double l = act[r] ? v[r][jj] * rp : 0.0;
                v[r][jj] = act[r] ? l : v[r][jj];
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c > jj) v[r][c] = fma(-l, pr[c], v[r][c]);
            }
        }
    }
}

// ------------------------------------------------------------------ LU, no interchanges
//
// Partial pivoting chooses the diagonal entry as the pivot of column c
// exactly when no entry below it is larger in magnitude, i.e. when every
// multiplier of the column satisfies |l| <= 1.  For block diagonally
// dominant systems this holds at every column, and the factorisation is
// then an LU without row interchanges, which needs no pivot search: the
// M x M block (M a multiple of 32, at most 256) is factored right-looking
// in 32-column panels:
//   D  one wave factors the 32 x 32 diagonal block A11 (one row per lane,
//      the pivot row read from its lane) and inverts L11 and U11 (the
//      four 16 x 16 diagonal blocks by forward substitution, a lane per
//      column, the two off-diagonal blocks on MFMA);
//   P  L21 = A21 inv(U11) and U12 = inv(L11) A12 on MFMA (all waves);
//   U  A22 -= L21 U12 on MFMA, two 16 x 16 tiles per wave at a time.
// It also leaves the factors prepared for the blocked triangular solves
// (what k_diag_prep does otherwise): inv(L11) and inv(U11) of every
// diagonal block into DI, the blocks below each diagonal block stored as
// L21 inv(L11) (one more product per panel task, L21 read back from LDS)
// and those above it as U12 inv(U11) (panel tasks of the next iteration,
// and of a last pass for the last block).
// Every pivot is checked to be finite and non-zero and every multiplier
// to satisfy |l| <= 1; if any check fails the factorisation is abandoned
// and the block is factored with interchanges from its unchanged working
// copy (the fast path reads the working copy and writes only the factor
// array).  On success the factors are those of partial pivoting with the
// identity permutation.
constexpr int NP_NB = 32, NP_TP = 33, NP_LPP = 33, NP_UPP = 228;

struct NpLds {
    size_t t11, f11, il, iu, ds, lp, up, flag, total;
};

// t11: the factored diagonal block, f11 the same block flipped; il, iu:
// inv(L11), inv(U11); ds: 32 ones, then the reciprocals of the diagonal of
// U11 in the order of its flipped 16 x 16 blocks; lp: L21 (rows below the block x 32);
// up: U12 (32 x columns right of the block); flag: failure of a check.
__host__ __device__ constexpr NpLds np_lds_layout() {
    NpLds l{};
    size_t off = 0;
    l.t11 = off; off += sizeof(double) * NP_NB * NP_TP;
    l.il = off; off += sizeof(double) * NP_NB * NP_TP;
    l.iu = off; off += sizeof(double) * NP_NB * NP_TP;
    l.ds = off; off += sizeof(double) * 2 * NP_NB;
    l.f11 = off; off += sizeof(double) * NP_NB * NP_TP;
    l.lp = off; off += sizeof(double) * (256 - NP_NB) * NP_LPP;
    l.up = off; off += sizeof(double) * NP_NB * NP_UPP;
    l.flag = off; off += 16;
    l.total = off;
    return l;
}
static_assert(np_lds_layout().total <= 160 * 1024, "no-interchange LU must fit the LDS");

// Phase D on one wave: factor A11 (rows j0.. of src, columns j0..) into T and
// out, inverses into IL and IU.  Returns this lane's checks.
__device__ __forceinline__ bool np_diag(const double* __restrict__ src, double* __restrict__ out, int M, int j0,
                                        double* T, double* F, double* IL, double* IU, double* DS, int lane) {
    constexpr int TP = NP_TP;
    const bool rowl = lane < 32;
    const int r = lane & 31;
    double v[32];
    const double* srow = src + (size_t)(j0 + r) * M + j0;
#pragma unroll
    for (int c = 0; c < 32; c += 2) {
        const double2 x = *(const double2*)(srow + c);
        v[c] = x.x;
        v[c + 1] = x.y;
    }
    bool ok = true;
    // every lane's reciprocal of its own entry in the next pivot column; the
    // pivot's lane holds the one needed
    auto recip = [](double x) {
        double rc = __builtin_amdgcn_rcp(x);
        rc = fma(rc, fma(-x, rc, 1.0), rc);
        return fma(rc, fma(-x, rc, 1.0), rc);
    };
    double rcv = recip(v[0]);
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        // the lane index made opaque per step: the step's lane masks are
        // formed here, not all 64 of them up front (scalar register pressure)
        int ln = lane;
        __asm__ volatile("" : "+v"(ln));
        // the pivot row and its reciprocal read straight from lane c (no
        // LDS round trip on the chain of column steps)
        const double pv = readlane_d(v[c], c);
        const double rp = readlane_d(rcv, c);
        ok = ok && pv != 0.0 && isfinite(pv);
        const bool act = ln < 32 && (ln & 31) > c;
        const double l = v[c] * rp;
        ok = ok && (!act || fabs(l) <= 1.0);
        // rows above get a zero multiple (a non-finite pivot row fails the
        // checks later on) and keep their values
        const double le = act ? l : 0.0;
        v[c] = act ? l : v[c];
        if (c + 1 < 32) {
            // the next pivot column first, and its reciprocal
            v[c + 1] = fma(-le, readlane_d(v[c + 1], c), v[c + 1]);
            rcv = recip(v[c + 1]);
        }
#pragma unroll
        for (int q = 0; q < 32; ++q)
            if (q > c + 1) v[q] = fma(-le, readlane_d(v[q], c), v[q]);
    }
    // the factored rows (multipliers left of the diagonal, U from it) to
    // T and out, and the block flipped, F[a][b] = T[31-a][31-b], whose lower
    // triangle is U11 reversed
    if (rowl) {
        double* orow = out + (size_t)(j0 + r) * M + j0;
#pragma unroll
        for (int q = 0; q < 32; q += 2) {
            T[r * TP + q] = v[q];
            T[r * TP + q + 1] = v[q + 1];
            *(double2*)(orow + q) = make_double2(v[q], v[q + 1]);
            F[(31 - r) * TP + 31 - q] = v[q];
            F[(31 - r) * TP + 30 - q] = v[q + 1];
        }
    }
    wave_lds_sync();
    // reciprocals of the diagonal of U11, in the order of the flipped blocks
    if (rowl) {
        DS[r] = 1.0;
        DS[r < 16 ? 32 + 15 - r : 48 + 31 - r] = 1.0 / T[r * TP + r];
    }
    wave_lds_sync();
    // The inverses in 16 x 16 blocks.  Lane group k = lane >> 4 inverts one
    // diagonal block by forward substitution, lane j its column j: k = 0, 1
    // the unit lower blocks L1 = L11[0:16, 0:16], L2 = L11[16:32, 16:32] (in
    // T); k = 2, 3 the upper blocks U1 = U11[0:16, 0:16], U2 = U11[16:32,
    // 16:32] through their flips U'[a][b] = U[15-a][15-b], lower triangles of
    // F, with inv(U)[15-a][j] = inv(U')[a][15-j].
    const int k4 = lane >> 4, j16 = lane & 15;
    const bool uk = k4 >= 2;
    const double* Mk = (k4 & 1) ? (uk ? F : T + 16 * TP + 16) : (uk ? F + 16 * TP + 16 : T);
    const double* Dk = DS + 16 * k4;
    const int jt = uk ? 15 - j16 : j16;
    // right-looking: once x[b] is final, it is removed from every later
    // row's sum (a dependent chain of one product per step; the loads of a
    // column do not wait for x)
    double x[16];
    {
        int jo = jt;
        __asm__ volatile("" : "+v"(jo));
#pragma unroll
        for (int a = 0; a < 16; ++a) x[a] = a == jo ? 1.0 : 0.0;
    }
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        x[b] *= Dk[b];
#pragma unroll
        for (int a = 0; a < 16; ++a)
            if (a > b) x[a] = fma(-Mk[a * TP + b], x[b], x[a]);
    }
    {
        const int ro = (k4 & 1) * 16;
#pragma unroll
        for (int a = 0; a < 16; ++a) {
            double* d = uk ? IU + (ro + 15 - a) * TP + ro + j16 : IL + (ro + a) * TP + ro + j16;
            *d = x[a];
        }
        // the zero blocks: inv(L11)[0:16, 16:32] (group 0), inv(U11)[16:32, 0:16] (group 3)
        if (k4 == 0 || k4 == 3) {
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                double* z = k4 == 0 ? IL + a * TP + 16 + j16 : IU + (16 + a) * TP + j16;
                *z = 0.0;
            }
        }
    }
    wave_lds_sync();
    // the off-diagonal blocks on MFMA:
    //   inv(L11)[16:32, 0:16] = -inv(L2) (L11[16:32, 0:16] inv(L1)),
    //   inv(U11)[0:16, 16:32] = -inv(U1) (U11[0:16, 16:32] inv(U2));
    // a product's output register v of lane group g holds row g + 4v, which
    // is the right operand of slice v of the next product as it stands
    {
        const int g = lane >> 4, cc = lane & 15;
        v4d y = {0.0, 0.0, 0.0, 0.0}, yu = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            y = mfma4(T[(16 + cc) * TP + 4 * kk + g], IL[(4 * kk + g) * TP + cc], y);
            yu = mfma4(T[cc * TP + 16 + 4 * kk + g], IU[(16 + 4 * kk + g) * TP + 16 + cc], yu);
        }
        v4d z = {0.0, 0.0, 0.0, 0.0}, zu = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            z = mfma4(IL[(16 + cc) * TP + 16 + 4 * kk + g], y[kk], z);
            zu = mfma4(IU[cc * TP + 4 * kk + g], yu[kk], zu);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            IL[(16 + g + 4 * v) * TP + cc] = -z[v];
            IU[(g + 4 * v) * TP + 16 + cc] = -zu[v];
        }
    }
    return ok;
}

// Two 16 x 16 tiles (t0, u0), (t1, u1) of the trailing matrix right of and
// below the diagonal block at j0: A22 -= L21 U12 (L21, U12 in LDS), read from
// src, written to out; the second tile is stored only if `second`.
__device__ __forceinline__ void np_tiles(const double* __restrict__ src, double* __restrict__ out, int M, int j0,
                                         int g, int cc, const double* LP, const double* UP, int t0, int u0, int t1,
                                         int u1, bool second) {
    constexpr int LPP = NP_LPP, UPP = NP_UPP;
    const double* cbase = src + (size_t)(j0 + NP_NB) * M + j0 + NP_NB;
    double* obase = out + (size_t)(j0 + NP_NB) * M + j0 + NP_NB;
    v4d c0, c1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        c0[v] = cbase[(size_t)(16 * t0 + g + 4 * v) * M + 16 * u0 + cc];
        c1[v] = cbase[(size_t)(16 * t1 + g + 4 * v) * M + 16 * u1 + cc];
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const double b0 = UP[(4 * kk + g) * UPP + 16 * u0 + cc];
        const double b1 = UP[(4 * kk + g) * UPP + 16 * u1 + cc];
        c0 = mfma4(-LP[(16 * t0 + cc) * LPP + 4 * kk + g], b0, c0);
        c1 = mfma4(-LP[(16 * t1 + cc) * LPP + 4 * kk + g], b1, c1);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) obase[(size_t)(16 * t0 + g + 4 * v) * M + 16 * u0 + cc] = c0[v];
    if (second) {
#pragma unroll
        for (int v = 0; v < 4; ++v) obase[(size_t)(16 * t1 + g + 4 * v) * M + 16 * u1 + cc] = c1[v];
    }
}

// The 2 x 2 tiles (t, u), (t, u+1), (t+1, u), (t+1, u+1) of the trailing
// matrix: A22 -= L21 U12 with each K slice's two L21 and two U12 operands
// read once for four products.
__device__ __forceinline__ void np_block(const double* __restrict__ src, double* __restrict__ out, int M, int j0,
                                         int g, int cc, const double* LP, const double* UP, int t, int u) {
    constexpr int LPP = NP_LPP, UPP = NP_UPP;
    const double* cbase = src + (size_t)(j0 + NP_NB) * M + j0 + NP_NB;
    double* obase = out + (size_t)(j0 + NP_NB) * M + j0 + NP_NB;
    v4d c[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) c[a][b][v] = cbase[(size_t)(16 * (t + a) + g + 4 * v) * M + 16 * (u + b) + cc];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        const double a0 = -LP[(16 * t + cc) * LPP + 4 * kk + g];
        const double a1 = -LP[(16 * (t + 1) + cc) * LPP + 4 * kk + g];
        const double b0 = UP[(4 * kk + g) * UPP + 16 * u + cc];
        const double b1 = UP[(4 * kk + g) * UPP + 16 * (u + 1) + cc];
        c[0][0] = mfma4(a0, b0, c[0][0]);
        c[0][1] = mfma4(a0, b1, c[0][1]);
        c[1][0] = mfma4(a1, b0, c[1][0]);
        c[1][1] = mfma4(a1, b1, c[1][1]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) obase[(size_t)(16 * (t + a) + g + 4 * v) * M + 16 * (u + b) + cc] = c[a][b][v];
}

// The no-interchange factorisation of one block; false (nothing but out
// written) when a check fails.  Called by all threads of the LU workgroup.
// inv(L11), inv(U11) of diagonal block b (in LDS, pitch NP_TP) to DI (all threads).
__device__ __forceinline__ void np_copy_inverses(const double* IL, const double* IU, double* __restrict__ di, int b,
                                                 int tid) {
    for (int idx = tid; idx < 2 * NP_NB * NP_NB; idx += LW_NT) {
        const int which = idx >> 10, r = (idx >> 5) & 31, c = idx & 31;
        di[(size_t)b * DI_STRIDE + which * NP_NB * NP_NB + r * NP_NB + c] = (which ? IU : IL)[r * NP_TP + c];
    }
}

// Rows [0, j0) of the block column at j0 of U (final U12 blocks of earlier
// panels) times inv(U11) of the diagonal block at j0 (32 x 32, row-major in
// global memory), in place; 16-row tasks k, k + nw, ... of this wave.
__device__ __forceinline__ void np_scale_u(double* __restrict__ out, const double* __restrict__ iu, int M, int j0,
                                           int g, int cc, int k, int nw) {
    for (int q = k; q < j0 / 16; q += nw) {
        const double* arow = out + (size_t)(16 * q + cc) * M + j0 + g;
        double av[8], b0[8], b1[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            av[kk] = arow[4 * kk];
            b0[kk] = iu[(4 * kk + g) * NP_NB + cc];
            b1[kk] = iu[(4 * kk + g) * NP_NB + 16 + cc];
        }
        v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            acc0 = mfma4(av[kk], b0[kk], acc0);
            acc1 = mfma4(av[kk], b1[kk], acc1);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double* orow = out + (size_t)(16 * q + g + 4 * v) * M + j0;
            orow[cc] = acc0[v];
            orow[16 + cc] = acc1[v];
        }
    }
}

__device__ __forceinline__ bool getrf_nointerchange(const double* __restrict__ a, double* __restrict__ out, int* __restrict__ perm,
                                    double* __restrict__ di, int M, char* smc) {
    constexpr NpLds lay = np_lds_layout();
    constexpr int TP = NP_TP, LPP = NP_LPP, UPP = NP_UPP;
    // array offsets kept in registers: every LDS access is then a register
    // base plus an immediate, instead of one scalar address constant per
    // access of the unrolled code (scalar register pressure)
    int off[7] = {(int)(lay.t11 / 8), (int)(lay.f11 / 8), (int)(lay.il / 8), (int)(lay.iu / 8),
                  (int)(lay.ds / 8), (int)(lay.lp / 8), (int)(lay.up / 8)};
#pragma unroll
    for (int k = 0; k < 7; ++k) __asm__ volatile("" : "+v"(off[k]));
    double* sd = (double*)smc;
    double* T = sd + off[0];
    double* F = sd + off[1];
    double* IL = sd + off[2];
    double* IU = sd + off[3];
    double* DS = sd + off[4];
    double* LP = sd + off[5];
    double* UP = sd + off[6];
    int* FL = (int*)(smc + lay.flag);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    constexpr int NW = LW_NT / 64;
    if (tid == 0) FL[0] = 0;
    __syncthreads();
    // Iteration j0 = -32 factors only the first diagonal block; iteration
    // j0 >= 0 forms L21, U12 of the block at j0, updates the next diagonal
    // block, then factors it (wave 0) while the other waves update the rest
    // of the trailing matrix.  One call site of np_diag (code size, registers).
    for (int j0 = -NP_NB; j0 + NP_NB < M; j0 += NP_NB) {
        const double* src = j0 <= 0 ? a : out;   // the trailing matrix: the working copy, then out
        const int m2 = M - j0 - NP_NB;            // rows below = columns right of the block
        // per-lane offsets made opaque per panel, so that the products' lane
        // addresses are not hoisted out of the loop and kept live across the
        // diagonal block (register pressure)
        int lv = lane;
        __asm__ volatile("" : "+v"(lv));
        const int g = lv >> 4, cc = lv & 15;
        const int nt2 = m2 / 16;
        if (j0 >= 0) {
            // ---- P: L21 = A21 inv(U11) by 16-row blocks (tasks q < nt2) and
            // U12 = inv(L11) A12 by 16-column blocks; a task reads all 32 columns
            // (rows) of its block before it overwrites them (in place from the
            // second panel on), so no two tasks share a block
            bool okp = true;
            // tasks q < nt2: rows of A21; nt2 <= q < 2 nt2: columns of A12.
            // A task's eight operands per lane (a row piece, or a column piece
            // of A12) are addressed without a branch; the next task's
            // operands are loaded before the current task's products (past
            // the last task: the last one again, unused).  The block's
            // inverses also go to DI (the rows of U above the block are
            // scaled from there during the update phase).
            const int nq = 2 * nt2;
            np_copy_inverses(IL, IU, di, j0 / NP_NB, tid);
            auto tload = [&](int q, double (&x)[8]) {
                const bool lt = q < nt2;
                const double* base = lt ? src + (size_t)(j0 + NP_NB + 16 * q + cc) * M + j0 + g
                                        : src + (size_t)(j0 + g) * M + j0 + NP_NB + 16 * (q - nt2) + cc;
                const size_t st = lt ? 4 : (size_t)4 * M;
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) x[kk] = base[kk * st];
            };
            double xv[8];
            if (w < nq) tload(w, xv);
            for (int q = w; q < nq; q += NW) {
                double xn[8];
                tload(min(q + NW, nq - 1), xn);
                v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
                if (q < nt2) {
                    const double* av = xv;
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk) {
                        acc0 = mfma4(av[kk], IU[(4 * kk + g) * TP + cc], acc0);
                        acc1 = mfma4(av[kk], IU[(4 * kk + g) * TP + 16 + cc], acc1);
                    }
                    {
                        // L21 to LP for the trailing update, L21 inv(L11) to out
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = 16 * q + g + 4 * v;
                            okp = okp && fabs(acc0[v]) <= 1.0 && fabs(acc1[v]) <= 1.0;
                            LP[row * LPP + cc] = acc0[v];
                            LP[row * LPP + 16 + cc] = acc1[v];
                        }
                        wave_lds_sync();
                        v4d s0 = {0.0, 0.0, 0.0, 0.0}, s1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int kk = 0; kk < 8; ++kk) {
                            const double l = LP[(16 * q + cc) * LPP + 4 * kk + g];
                            s0 = mfma4(l, IL[(4 * kk + g) * TP + cc], s0);
                            s1 = mfma4(l, IL[(4 * kk + g) * TP + 16 + cc], s1);
                        }
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            double* orow = out + (size_t)(j0 + NP_NB + 16 * q + g + 4 * v) * M + j0;
                            orow[cc] = s0[v];
                            orow[16 + cc] = s1[v];
                        }
                    }
                } else {
                    const int u = q - nt2;
                    const double* bv = xv;
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk) {
                        acc0 = mfma4(IL[cc * TP + 4 * kk + g], bv[kk], acc0);
                        acc1 = mfma4(IL[(16 + cc) * TP + 4 * kk + g], bv[kk], acc1);
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = g + 4 * v, col = 16 * u + cc;
                        out[(size_t)(j0 + row) * M + j0 + NP_NB + col] = acc0[v];
                        out[(size_t)(j0 + 16 + row) * M + j0 + NP_NB + col] = acc1[v];
                        UP[row * UPP + col] = acc0[v];
                        UP[(16 + row) * UPP + col] = acc1[v];
                    }
                }
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) xv[kk] = xn[kk];
            }
            if (__ballot(!okp) != 0ull && lane == 0) FL[0] = 1;
            __syncthreads();
            if (FL[0]) return false;
        }
        // ---- U: A22 -= L21 U12.  The next diagonal block's four tiles
        // first (waves 0-1); then wave 0 factors that block while waves 1-7
        // update the other tiles, two at a time (two MFMA chains).
        if (j0 >= 0) {
            // the 2 x 2 tiles of the next diagonal block
            if (w < 2) np_tiles(src, out, M, j0, g, cc, LP, UP, w, 0, w, 1, true);
            __syncthreads();
        }
        if (w == 0) {
            const bool ok = np_diag(j0 < 0 ? a : out, out, M, j0 + NP_NB, T, F, IL, IU, DS, lane);
            if (__ballot(!ok) != 0ull && lane == 0) FL[0] = 1;
        } else if (j0 >= 0) {
            // the other tiles in 2 x 2 blocks (the block of the next diagonal
            // block excluded): two row operands and two column operands from
            // LDS feed four products per K slice
            const int nb2 = nt2 / 2;
            for (int kb = w; kb < nb2 * nb2; kb += NW - 1) {
                const int bt = kb / nb2, bu = kb - bt * nb2;
                np_block(src, out, M, j0, g, cc, LP, UP, 2 * bt, 2 * bu);
            }
            // the rows of U above the block at j0 scaled by its inv(U11)
            // (read from DI: wave 0 is replacing the LDS copy), beside the
            // diagonal block's factorisation
            np_scale_u(out, di + (size_t)(j0 / NP_NB) * DI_STRIDE + NP_NB * NP_NB, M, j0, g, cc, w - 1, NW - 1);
        }
        __syncthreads();
        if (FL[0]) return false;
    }
    // the last diagonal block: its inverses, and the rows of U above it scaled
    {
        const int jl = M - NP_NB;
        np_copy_inverses(IL, IU, di, jl / NP_NB, tid);
        __syncthreads();
        int lv = lane;
        __asm__ volatile("" : "+v"(lv));
        np_scale_u(out, di + (size_t)(jl / NP_NB) * DI_STRIDE + NP_NB * NP_NB, M, jl, lv >> 4, lv & 15, w, NW);
    }
    for (int q = tid; q < M; q += LW_NT) perm[q] = q;
    return true;
}

__device__ void diag_prep_row_lw(const Level& L, int i, double* lds);

__global__ __launch_bounds__(LW_NT) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_getrf_pw(const KArgs ka) {
    constexpr int NB = LW_NB, P = LW_P;
    const Level& L = ka.L;
    const int kch = ka.c0 + blockIdx.x, t = ka.step;
    const int r0 = chunk_first(L, kch), e = chunk_last(L, kch);
    if (t > e - r0) return;
    const int i = r0 + t;
    const int M = L.M;
    const int tid = threadIdx.x, lane0 = tid & 63, w = tid >> 6;
    double* a = L.Dw + (size_t)kch * M * M;      // working copy, rows in place
    double* out = L.LU + (size_t)i * M * M;      // factors, rows in pivot order
    int* perm = L.perm + (size_t)i * M;
    // at a chunk's first row D_i = A_i: no forward product runs at that
    // step, so the factorisation reads A_i itself (the pivoting path, which
    // works in place, copies it into the working copy first)
    const double* a_in = t == 0 ? L.A + (size_t)i * M * M : a;
    extern __shared__ double sm_raw[];
    char* smc = (char*)sm_raw;
    // the case without row interchanges first (it also prepares the factors
    // for the triangular solves); the factorisation with interchanges below
    // when a check of it fails
    if ((M & (NP_NB - 1)) == 0 &&
        getrf_nointerchange(a_in, out, perm, L.DI + (size_t)i * (M / DB) * DI_STRIDE, M, smc))
        return;
    if (t == 0)
        for (int q = tid; q < M * M; q += LW_NT) a[q] = a_in[q];
    __syncthreads();   // its LDS is reused (and the working copy complete)
    constexpr LwLds lay = lw_lds_layout();
    double* NX = (double*)(smc + lay.nx);
    double* LB = (double*)(smc + lay.lb);
    double* TB = (double*)(smc + lay.tb);
    double* UN = (double*)(smc + lay.un);
    int* LIST = (int*)(smc + lay.list);
    int* PIV = (int*)(smc + lay.piv);
    double* PROW = (double*)(smc + lay.prow);
    const int npan = (M + NB - 1) / NB;

    // the columns of panels 0 and 1 of every row
    for (int idx = tid; idx < 2 * 256 * NB; idx += LW_NT) {
        const int b = idx / (256 * NB), rem = idx % (256 * NB), row = rem / NB, c = rem % NB;
        const int col = b * NB + c;
        NX[(b * 256 + row) * P + c] = (row < M && col < M) ? a[(size_t)row * M + col] : 0.0;
    }
    __syncthreads();

    bool act[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) act[r] = w == 0 && 4 * lane0 + r < M;
    int fail_code = 0, fail_col = -1;
    int p = 0;
    for (;; ++p) {
        int lv = lane0;
        __asm__ volatile("" : "+v"(lv));   // keep per-lane addresses from being hoisted out of the loop
        const int lane = lv, g = lv >> 4, cc = lv & 15;
        const int j0 = p * NB, nb = min(NB, M - j0);
        const int w2 = M - j0 - nb;          // columns right of panel p = rows left after it
        const int cur = p & 1, nxt = cur ^ 1;
        if (w == 0) {
            // ---------------- panel p
            double v[4][NB];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < NB; ++c) v[r][c] = act[r] ? NX[(cur * 256 + 4 * lane + r) * P + c] : 0.0;
            bool act0[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) act0[r] = act[r];
            lw_panel_steps(v, act, fail_code, fail_col, j0, nb, lane, PIV + cur * NB, PROW);
            // publish the panel rows and the list of rows left (row order)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (act0[r]) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) LB[(cur * 256 + 4 * lane + r) * P + c] = v[r][c];
                }
            int pos = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const unsigned long long bal = __ballot(act[r]);
                pos += __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (act[r]) LIST[cur * 256 + pos++] = 4 * lane + r;
        } else if (p > 0) {
            // ---------------- panel q = p-1 applied right of panel p; its factor rows
            const int q = p - 1, qc = q & 1, j0q = q * NB;
            const int hq = M - j0q - NB;                 // rows left after panel q
            const int cs0 = j0 + NB;                     // first column right of panel p
            const int nsl = cs0 < M ? (M - cs0 + NB - 1) / NB : 0;
            const int* pvq = PIV + qc * NB;
            const int* lsq = LIST + qc * 256;
            const double* lbq = LB + (size_t)qc * 256 * P;
            double* nxd = NX + (size_t)nxt * 256 * P;   // columns of panel p+1
            // Every load below is unconditional, from a clamped address (row 0
            // or column 0 for the rows and columns outside the update), so that
            // the loop has no divergent branches: the loads of one 64-row batch
            // stay in flight while the previous batch is multiplied.  Entries
            // of rows or columns outside the update are never stored, and a
            // tile row or column does not reach any other in the product.
            for (int s = w - 1; s < nsl; s += LW_HW) {
                const int col = cs0 + s * NB + cc;
                const bool cok = col < M;
                const int cs = cok ? col : 0;
                double bo[4];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) bo[kk] = a[(size_t)pvq[4 * kk + g] * M + cs];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) bo[kk] = cok ? bo[kk] : 0.0;
                v4d u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) u = mfma4(TB[cc * P + 4 * kk + g], bo[kk], u);
#pragma unroll
                for (int vv = 0; vv < 4; ++vv)
                    if (cok) out[(size_t)(j0q + g + 4 * vv) * M + col] = u[vv];
                // A22 -= L21 U12 over the rows left, four 16-row tiles per
                // batch; hq <= 240, so a batch index stays below 256
                const int nbt = (hq + 63) / 64;
                auto load_batch = [&](int tb, v4d (&c)[4], int (&rw)[4][4]) {
#pragma unroll
                    for (int x = 0; x < 4; ++x)
#pragma unroll
                        for (int vv = 0; vv < 4; ++vv) {
                            const int idx = tb + 16 * x + g + 4 * vv;
                            const int lv = lsq[idx];
                            rw[x][vv] = idx < hq ? lv : -1;
                        }
#pragma unroll
                    for (int x = 0; x < 4; ++x)
#pragma unroll
                        for (int vv = 0; vv < 4; ++vv)
                            c[x][vv] = a[(uint32_t)(max(rw[x][vv], 0) * M + cs)];
                };
                auto mul_store = [&](int tb, v4d (&c)[4], const int (&rw)[4][4]) {
                    double ao[4][4];
#pragma unroll
                    for (int x = 0; x < 4; ++x) {
                        const int ai = tb + 16 * x + cc;
                        const int lv = lsq[ai];
                        const int ar = ai < hq ? lv : -1;
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) {
                            const double l = lbq[max(ar, 0) * P + 4 * kk + g];
                            ao[x][kk] = ar >= 0 ? -l : 0.0;
                        }
                    }
#pragma unroll
                    for (int x = 0; x < 4; ++x)
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) c[x] = mfma4(ao[x][kk], u[kk], c[x]);
#pragma unroll
                    for (int x = 0; x < 4; ++x)
#pragma unroll
                        for (int vv = 0; vv < 4; ++vv)
                            if (rw[x][vv] >= 0 && cok) {
                                if (s == 0) nxd[rw[x][vv] * P + cc] = c[x][vv];
                                else a[(uint32_t)(rw[x][vv] * M + col)] = c[x][vv];
                            }
                };
                v4d c0[4], c1[4];
                int r0[4][4], r1[4][4];
                load_batch(0, c0, r0);
                for (int bt = 0; bt < nbt; bt += 2) {
                    // the batch after this one (the last one again at the end, unused)
                    load_batch(min(bt + 1, nbt - 1) * 64, c1, r1);
                    mul_store(bt * 64, c0, r0);
                    if (bt + 1 >= nbt) break;
                    load_batch(min(bt + 2, nbt - 1) * 64, c0, r0);
                    mul_store((bt + 1) * 64, c1, r1);
                }
            }
            // factor rows of panel q: the multipliers left of the panel from the
            // working copy (eight loads in flight per lane), the panel from LDS,
            // the next panel's U12; the pivot order; the multipliers of the rows
            // left back to the working copy
            const int hs = (w - 1) * 64 + lane;
            const int n0 = NB * j0q;
            for (int base = hs; base < n0; base += 8 * LW_HW * 64) {
                double val[8];
#pragma unroll
                for (int u8 = 0; u8 < 8; ++u8) {
                    const int x = base + u8 * LW_HW * 64, rr = x / j0q, c = x - rr * j0q;
                    val[u8] = x < n0 ? a[(size_t)pvq[rr] * M + c] : 0.0;
                }
#pragma unroll
                for (int u8 = 0; u8 < 8; ++u8) {
                    const int x = base + u8 * LW_HW * 64, rr = x / j0q, c = x - rr * j0q;
                    if (x < n0) out[(size_t)(j0q + rr) * M + c] = val[u8];
                }
            }
            const int W1 = min(M - j0q, NB + nb);   // panel q and the next panel's columns
            const int n1 = NB * W1, n2 = hq * NB;
            for (int x = hs; x < n1 + n2; x += LW_HW * 64) {
                if (x < n1) {
                    const int rr = x / W1, c = x - rr * W1;
                    const int prow = pvq[rr];
                    out[(size_t)(j0q + rr) * M + j0q + c] = c < NB ? lbq[prow * P + c] : UN[rr * P + c - NB];
                    if (c == 0) perm[j0q + rr] = prow;
                } else {
                    const int y = x - n1, ri = y / NB, c = y - ri * NB;
                    const int row = lsq[ri];
                    a[(size_t)row * M + j0q + c] = lbq[row * P + c];
                }
            }
        }
        __syncthreads();   // panel p published; panel p-1 applied
        if (w2 <= 0) break;
        const int nb2 = min(NB, w2);
        // ---------------- inv(L11) of panel p and U12 of the columns of panel p+1
        if (w == 0) {
            const int* pv = PIV + cur * NB;
            const double* lb = LB + (size_t)cur * 256 * P;
            if (lane < NB) {
                const int jc = lane;
                double x[NB];
#pragma unroll
                for (int rr = 0; rr < NB; ++rr) {
                    const double* lr = lb + pv[rr] * P;
                    double s4[4] = {rr == jc ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int c = 0; c < rr; ++c) s4[c & 3] = fma(-lr[c], x[c], s4[c & 3]);
                    x[rr] = rr >= jc ? (s4[0] + s4[1]) + (s4[2] + s4[3]) : 0.0;
                }
#pragma unroll
                for (int rr = 0; rr < NB; ++rr) TB[rr * P + jc] = x[rr];
            }
            wave_lds_sync();
            const double* nxn = NX + (size_t)nxt * 256 * P;
            v4d acc = {0.0, 0.0, 0.0, 0.0};
            double bn[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const double x = nxn[pv[4 * kk + g] * P + cc];   // cc < 16 < P: inside the row
                bn[kk] = cc < nb2 ? x : 0.0;
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) acc = mfma4(TB[cc * P + 4 * kk + g], bn[kk], acc);
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) UN[(g + 4 * vv) * P + cc] = acc[vv];
        }
        __syncthreads();
        // ---------------- the columns of panel p+1 of the rows left: -= L21 U12 (all waves)
        {
            const double* lb = LB + (size_t)cur * 256 * P;
            const int* ls = LIST + cur * 256;
            double* nxn = NX + (size_t)nxt * 256 * P;
            // reads from clamped LDS addresses (w2 <= 240, so every index
            // stays below 256), no divergent branch; rows outside are not stored
            for (int tb = w * 16; tb < w2; tb += 8 * 16) {
                int rw[4];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    const int idx = tb + g + 4 * vv;
                    const int lv = ls[idx];
                    rw[vv] = idx < w2 ? lv : -1;
                }
                v4d cv;
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) cv[vv] = nxn[max(rw[vv], 0) * P + cc];
                const int ai = tb + cc;
                const int lv = ls[ai];
                const int ar = ai < w2 ? lv : -1;
                double ao[4];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const double l = lb[max(ar, 0) * P + 4 * kk + g];
                    ao[kk] = ar >= 0 ? -l : 0.0;
                }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) cv = mfma4(ao[kk], UN[(4 * kk + g) * P + cc], cv);
#pragma unroll
                for (int vv = 0; vv < 4; ++vv)
                    if (rw[vv] >= 0) nxn[rw[vv] * P + cc] = cv[vv];
            }
        }
        __syncthreads();
    }
    // ---------------- factor rows of the last panel (eight loads in flight per
    // thread), the failure report
    {
        const int j0 = p * NB, nb = M - j0, cur = p & 1;
        const int* pv = PIV + cur * NB;
        const double* lb = LB + (size_t)cur * 256 * P;
        for (int base = tid; base < nb * M; base += 8 * LW_NT) {
            double val[8];
#pragma unroll
            for (int u8 = 0; u8 < 8; ++u8) {
                const int x = base + u8 * LW_NT, rr = x / M, c = x - rr * M;
                val[u8] = x < nb * M ? (c < j0 ? a[(size_t)pv[rr] * M + c] : lb[pv[rr] * P + c - j0]) : 0.0;
            }
#pragma unroll
            for (int u8 = 0; u8 < 8; ++u8) {
                const int x = base + u8 * LW_NT, rr = x / M, c = x - rr * M;
                if (x < nb * M) {
                    out[(size_t)(j0 + rr) * M + c] = val[u8];
                    if (c == 0) perm[j0 + rr] = pv[rr];
                }
            }
        }
    }
    if (w == 0 && lane0 == 0 && fail_code != 0) report_status(ka.status, L.level, i, fail_col, fail_code);
    // for M a multiple of 32 no separate preparation follows (the case
    // without interchanges prepares its rows): prepare this row here
    if ((M & (NP_NB - 1)) == 0) {
        __syncthreads();   // the factors are written, the LDS is free
        diag_prep_row_lw(L, i, sm_raw);
    }
}

// Preparation of the factors of every D_i factored at this step for the
// blocked triangular solves, one 256-thread workgroup per (32-column block
// b, chunk):
//   * the inverses of the diagonal blocks inv(L_bb) (unit lower) and
//     inv(U_bb), padded with the identity past the end of the matrix, into DI;
//   * the off-diagonal blocks of block column b scaled in place by them:
//     L_{b',b} := L_{b',b} inv(L_bb) below the diagonal block and
//     U_{b',b} := U_{b',b} inv(U_bb) above it (MFMA).
// With the scaled blocks a sweep updates the other rows with the block
// before its diagonal solve, so no diagonal product sits on the sweep's
// sequential chain: for L y = r, w_b = r_b - sum_{b'<b} Lt_{b,b'} w_{b'} and
// y_b = inv(L_bb) w_b; likewise for U.
// Block column bb of row i (all NT threads; blk and inv: LDS of
// DB (DB + 1) and 2 DB (DB + 1) doubles).
template <int NT>
__device__ __forceinline__ void diag_prep_block(const Level& L, int i, int bb, double* blk, double (*inv)[DB * (DB + 1)]) {
    const int M = L.M;
    const int b0 = bb * DB, bs = min(DB, M - b0);
    const int nblk = (M + DB - 1) / DB;
    double* a = L.LU + (size_t)i * M * M;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int idx = tid; idx < DB * DB; idx += NT) {
        const int rr = idx / DB, cc = idx % DB;
        blk[rr * (DB + 1) + cc] = (rr < bs && cc < bs) ? a[(size_t)(b0 + rr) * M + b0 + cc] : 0.0;
    }
    __syncthreads();
    if (tid < 2 * DB) {
        const int which = tid / DB, jc = tid % DB;
        double x[DB];
        if (which == 0) {
#pragma unroll
            for (int rr = 0; rr < DB; ++rr) {
                double s = (rr == jc) ? 1.0 : 0.0;
#pragma unroll
                for (int c = 0; c < rr; ++c) s = fma(-blk[rr * (DB + 1) + c], x[c], s);
                x[rr] = (rr < bs || rr == jc) ? s : 0.0;
            }
        } else {
#pragma unroll
            for (int rr = DB - 1; rr >= 0; --rr) {
                double s = (rr == jc) ? 1.0 : 0.0;
#pragma unroll
                for (int c = DB - 1; c > rr; --c) s = fma(-blk[rr * (DB + 1) + c], x[c], s);
                x[rr] = rr < bs ? s / blk[rr * (DB + 1) + rr] : ((rr == jc) ? 1.0 : 0.0);
            }
        }
        double* di = L.DI + (size_t)i * nblk * DI_STRIDE + (size_t)bb * DI_STRIDE + (which ? DB * DB : 0);
#pragma unroll
        for (int rr = 0; rr < DB; ++rr) {
            di[rr * DB + jc] = x[rr];
            inv[which][rr * (DB + 1) + jc] = x[rr];
        }
    }
    __syncthreads();
    // scale the off-diagonal blocks of this block column: 16-row strips, one wave each
    for (int st = w; st < 2 * nblk; st += NT / 64) {
        if (st / 2 == bb) continue;
        const int which = (st / 2 > bb) ? 0 : 1;
        const int row0 = st * 16;
        const int grow = row0 + (lane & 15);
        double av[DB / 4];
#pragma unroll
        for (int kk = 0; kk < DB / 4; ++kk) {
            const int gk = b0 + kk * 4 + (lane >> 4);
            av[kk] = (grow < M && gk < M) ? a[(size_t)grow * M + gk] : 0.0;
        }
        v4d acc[2];
#pragma unroll
        for (int tc = 0; tc < 2; ++tc) {
            acc[tc] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < DB / 4; ++kk)
                acc[tc] = mfma4(av[kk], inv[which][(kk * 4 + (lane >> 4)) * (DB + 1) + tc * 16 + (lane & 15)], acc[tc]);
        }
#pragma unroll
        for (int tc = 0; tc < 2; ++tc) {
            const int gc = b0 + tc * 16 + (lane & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = row0 + (lane >> 4) + 4 * v;
                if (row < M && gc < M) a[(size_t)row * M + gc] = acc[tc][v];
            }
        }
    }
}

// All block columns of row i from the LU kernel (its 512 threads, its LDS).
__device__ __forceinline__ void diag_prep_row_lw(const Level& L, int i, double* lds) {
    // the LDS offsets held in registers (not one scalar constant per access)
    int o1 = 0, o2 = DB * (DB + 1);
    __asm__ volatile("" : "+v"(o1), "+v"(o2));
    double* blk = lds + o1;
    double (*inv)[DB * (DB + 1)] = (double (*)[DB * (DB + 1)])(lds + o2);
#pragma nounroll
    for (int bb = 0; bb < L.M / DB; ++bb) {
        diag_prep_block<LW_NT>(L, i, bb, blk, inv);
        __syncthreads();
    }
}

// One workgroup per (block column, chunk), for block sizes whose LU does not
// prepare its rows itself (M not a multiple of 32, or above 256).
__global__ __launch_bounds__(256) void k_diag_prep(const KArgs ka) {
    const Level& L = ka.L;
    const int k = ka.c0 + blockIdx.y, t = ka.step;
    const int r0 = chunk_first(L, k), e = chunk_last(L, k);
    if (t > e - r0) return;
    __shared__ double blk[DB * (DB + 1)];
    __shared__ double inv[2][DB * (DB + 1)];
    diag_prep_block<256>(L, r0 + t, blockIdx.x, blk, inv);
}

// ------------------------------------------------------------------ triangular solves
//
// In place on the M x 2M right-hand side W_i = [C_i | -B_i Y_{i-1}]
// (row-major): X := U^{-1} L^{-1} (P X), one slab of SW columns per
// 256-thread workgroup, with the scaled off-diagonal blocks prepared by
// k_diag_prep.  The slab lives in MFMA accumulator registers: row block b
// (32 rows) belongs to wave b mod 4.  Each sweep step publishes the current
// (not yet diagonally solved) block b through a double-buffered LDS tile;
// after one barrier every wave subtracts Lt_{b',b} X_b (forward, b' > b) or
// Ut_{b',b} X_b (backward, b' < b) from its own blocks, with the operands of
// the next step already in flight.  After each sweep every wave applies the
// diagonal inverses to its own blocks.  Column validity is decided per
// column, so a slab can straddle the E and Y halves of W.
// The contraction index of the 32-wide block products is permuted so that
// lane group g = lane >> 4 takes k = 8 g + kk at MFMA step kk: each lane's
// eight operands of a row are then contiguous (two 32-byte loads) and the
// LDS operand of step kk is row 8 g + kk.
template <int SW, int BPW>
__device__ __forceinline__ void trsm_load_ops(const double* __restrict__ lu, int M, int nblk, int dir, int b, int w,
                                              int lane, double (&ops)[BPW][2][DB / 4]) {
    const int g = lane >> 4;
#pragma unroll
    for (int jb = 0; jb < BPW; ++jb) {
        const int bp = w + 4 * jb;
        const bool need = bp < nblk && (dir == 0 ? bp > b : bp < b);
#pragma unroll
        for (int tr = 0; tr < 2; ++tr) {
            const int grow = bp * DB + tr * 16 + (lane & 15);
            const int gk0 = b * DB + g * 8;
            if (need && grow < M && gk0 + 7 < M && (M & 3) == 0) {  // 32-byte aligned rows
                const double4* src = (const double4*)(lu + (size_t)grow * M + gk0);
                const double4 v0 = src[0], v1 = src[1];
                ops[jb][tr][0] = -v0.x; ops[jb][tr][1] = -v0.y; ops[jb][tr][2] = -v0.z; ops[jb][tr][3] = -v0.w;
                ops[jb][tr][4] = -v1.x; ops[jb][tr][5] = -v1.y; ops[jb][tr][6] = -v1.z; ops[jb][tr][7] = -v1.w;
            } else {
#pragma unroll
                for (int kk = 0; kk < DB / 4; ++kk) {
                    const int gk = gk0 + kk;
                    ops[jb][tr][kk] = (need && grow < M && gk < M) ? -lu[(size_t)grow * M + gk] : 0.0;
                }
            }
        }
    }
}

// X_jb := inv(T_bb) X_jb for all of this wave's blocks (dir 0: L, 1: U),
// through the wave's own LDS tile.
template <int SW, int BPW>
__device__ __forceinline__ void trsm_diag_own(const double* __restrict__ di, int nblk, int dir, int w, int lane,
                                              v4d (&x)[BPW][2][SW / 16], double* own) {
    constexpr int NSUB = SW / 16, PX = SW + 2;
#pragma unroll
    for (int jb = 0; jb < BPW; ++jb) {
        const int b = w + 4 * jb;
        if (b < nblk) {
            const double* inv = di + (size_t)b * DI_STRIDE + (dir == 0 ? 0 : DB * DB);
            double ia[2][DB / 4];
#pragma unroll
            for (int tr = 0; tr < 2; ++tr)
#pragma unroll
                for (int kk = 0; kk < DB / 4; ++kk) ia[tr][kk] = inv[(tr * 16 + (lane & 15)) * DB + kk * 4 + (lane >> 4)];
#pragma unroll
            for (int tr = 0; tr < 2; ++tr)
#pragma unroll
                for (int tc = 0; tc < NSUB; ++tc)
#pragma unroll
                    for (int v = 0; v < 4; ++v) own[(tr * 16 + (lane >> 4) + 4 * v) * PX + tc * 16 + (lane & 15)] = x[jb][tr][tc][v];
            wave_lds_sync();
#pragma unroll
            for (int tr = 0; tr < 2; ++tr)
#pragma unroll
                for (int tc = 0; tc < NSUB; ++tc) {
                    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int kk = 0; kk < DB / 4; ++kk)
                        acc = mfma4(ia[tr][kk], own[(kk * 4 + (lane >> 4)) * PX + tc * 16 + (lane & 15)], acc);
                    x[jb][tr][tc] = acc;
                }
            wave_lds_sync();
        }
    }
}

template <int SW, int BPW>
__device__ void getrs_slab(const double* __restrict__ lu, const double* __restrict__ di,
                           const int* __restrict__ perm, double* X, int ld, int M, int c0, int ncols, int valid_lo,
                           int valid_hi, int valid2_lo, int valid2_hi, double* xb /* 2 x [DB][SW+2] */,
                           double* ownb /* 4 x [DB][SW+2] */) {
    constexpr int NSUB = SW / 16;
    constexpr int PX = SW + 2;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nblk = (M + DB - 1) / DB;
    double* own = ownb + (size_t)w * DB * PX;
    PHASE_MARK(g_t0);
    auto valid = [&](int col) {
        return col < ncols && ((col >= valid_lo && col < valid_hi) || (col >= valid2_lo && col < valid2_hi));
    };
    // the slab, permuted (row indices staged in LDS), into accumulator registers
    int* sperm = (int*)(xb + 2 * DB * PX);
    for (int r = tid; r < M; r += 256) sperm[r] = perm[r];
    __syncthreads();
    v4d x[BPW][2][NSUB];
#pragma unroll
    for (int jb = 0; jb < BPW; ++jb)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int tc = 0; tc < NSUB; ++tc) {
                const int col = c0 + tc * 16 + (lane & 15);
                const bool cv = valid(col);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = (w + 4 * jb) * DB + tr * 16 + (lane >> 4) + 4 * v;
                    x[jb][tr][tc][v] = (row < M && cv) ? X[(size_t)sperm[row] * ld + col] : 0.0;
                }
            }
    double ops[BPW][2][DB / 4];
    trsm_load_ops<SW, BPW>(lu, M, nblk, 0, 0, w, lane, ops);
    int buf = 0;
    PHASE_MARK(g_t1);
    PHASE_ADD(5, g_t0, g_t1);
    for (int dir = 0; dir < 2; ++dir) {
        for (int step = 0; step < nblk; ++step) {
            const int b = dir == 0 ? step : nblk - 1 - step;
            double* xt = xb + (size_t)buf * DB * PX;
            if (w == (b & 3)) {
#pragma unroll
                for (int jb = 0; jb < BPW; ++jb)
                    if (jb == (b >> 2)) {
#pragma unroll
                        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
                            for (int tc = 0; tc < NSUB; ++tc)
#pragma unroll
                                for (int v = 0; v < 4; ++v)
                                    xt[(tr * 16 + (lane >> 4) + 4 * v) * PX + tc * 16 + (lane & 15)] = x[jb][tr][tc][v];
                    }
            }
            PHASE_MARK(g_b0);
            __syncthreads();
            PHASE_MARK(g_b1);
            PHASE_ADD(6, g_b0, g_b1);
            PHASE_ADD_W1(12, g_b0, g_b1);
            double cur[BPW][2][DB / 4];
#pragma unroll
            for (int jb = 0; jb < BPW; ++jb)
#pragma unroll
                for (int tr = 0; tr < 2; ++tr)
#pragma unroll
                    for (int kk = 0; kk < DB / 4; ++kk) cur[jb][tr][kk] = ops[jb][tr][kk];
            if (step + 1 < nblk) trsm_load_ops<SW, BPW>(lu, M, nblk, dir, dir == 0 ? step + 1 : nblk - 2 - step, w, lane, ops);
            else if (dir == 0) trsm_load_ops<SW, BPW>(lu, M, nblk, 1, nblk - 1, w, lane, ops);
            // the published block as B operands, read once for all of this wave's blocks
            double bo[NSUB][DB / 4];
#pragma unroll
            for (int tc = 0; tc < NSUB; ++tc)
#pragma unroll
                for (int kk = 0; kk < DB / 4; ++kk) bo[tc][kk] = xt[((lane >> 4) * 8 + kk) * PX + tc * 16 + (lane & 15)];
#pragma unroll
            for (int jb = 0; jb < BPW; ++jb) {
                const int bp = w + 4 * jb;
                if (bp < nblk && (dir == 0 ? bp > b : bp < b)) {
#pragma unroll
                    for (int kk = 0; kk < DB / 4; ++kk)
#pragma unroll
                        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
                            for (int tc = 0; tc < NSUB; ++tc)
                                x[jb][tr][tc] = mfma4(cur[jb][tr][kk], bo[tc][kk], x[jb][tr][tc]);
                }
            }
            buf ^= 1;
            PHASE_MARK(g_b2);
            PHASE_ADD(7, g_b1, g_b2);
            PHASE_ADD_W1(13, g_b1, g_b2);
        }
        // diagonal solves of this wave's blocks (off the sequential chain)
        PHASE_MARK(g_d0);
        trsm_diag_own<SW, BPW>(di, nblk, dir, w, lane, x, own);
        PHASE_MARK(g_d1);
        PHASE_ADD(10, g_d0, g_d1);
    }
#pragma unroll
    for (int jb = 0; jb < BPW; ++jb)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int tc = 0; tc < NSUB; ++tc) {
                const int col = c0 + tc * 16 + (lane & 15);
                const bool cv = valid(col);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = (w + 4 * jb) * DB + tr * 16 + (lane >> 4) + 4 * v;
                    if (row < M && cv) X[(size_t)row * ld + col] = x[jb][tr][tc][v];
                }
            }
    PHASE_MARK(g_t2);
    PHASE_ADD(11, g_t1, g_t2);
    PHASE_ADD(4, g_t0, g_t2);
}

// RHS = W_i = [C_i | -B_i Y_{i-1}] of chunk blockIdx.y at step t.
template <int SW, int BPW>
__global__ __launch_bounds__(256) void k_getrs(const KArgs ka) {
    __shared__ double xb[2 * DB * (SW + 2) + BTD_MAX_M / 2];  // two publish tiles + the row permutation
    __shared__ double ownb[4 * DB * (SW + 2)];
    const Level& L = ka.L;
    const int M = L.M, nslab = (2 * M + SW - 1) / SW;
    const int lid = xcd_logical_id(blockIdx.x, gridDim.x);
    const int k = ka.c0 + lid / nslab, t = ka.step;
    const int r = chunk_first(L, k), e = chunk_last(L, k);
    if (t > e - r) return;
    const int i = r + t;
    const int c0 = (lid % nslab) * SW;
    const int nblk = (M + DB - 1) / DB;
    const double* lu = L.LU + (size_t)i * M * M;
    const double* di = L.DI + (size_t)i * nblk * DI_STRIDE;
    const int* perm = L.perm + (size_t)i * M;
    const int e_lo = 0, e_hi = (i != L.N - 1) ? M : 0;
    const int y_lo = M, y_hi = (k > 0) ? 2 * M : M;
    const int c_end = c0 + SW;
    const bool any = (c0 < e_hi && c_end > e_lo) || (c0 < y_hi && c_end > y_lo);
    if (!any) return;
    getrs_slab<SW, BPW>(lu, di, perm, L.W + (size_t)i * M * M * 2, 2 * M, M, c0, 2 * M, e_lo, e_hi, y_lo, y_hi, xb,
                        ownb);
}

// ------------------------------------------------------------------ triangular solves, one slab per wave
//
// For M <= 256: X := U^{-1} L^{-1} (P X) on a slab of 16*NT16 columns of
// W_i, held entirely in one wave's MFMA accumulators.  With the scaled
// off-diagonal blocks of k_diag_prep a sweep subtracts Lt_{b',b} w_b
// (forward, b' > b) or Ut_{b',b} w_b (backward, b' < b) with the unsolved
// block w_b, and the diagonal inverses are applied to all blocks after each
// sweep.
//
// Register layout: in lane l (g = l >> 4, j = l & 15) accumulator register
// v of row tile tr of block b holds row 32b + 8g + 4tr + v, column j of
// the column tile.  Then the block product's contraction can run with lane
// group g taking k = 8g + kk at MFMA step kk (kk = 0..7): the right operand
// of step kk is this lane's own register (tile kk >> 2, register kk & 3),
// and the left operand (a block of the factors) is read as eight
// consecutive doubles per lane.  For output tile tr the left operand of
// lane l is row 8(i & 3) + 4tr + (i >> 2), i = l & 15, of the block.
template <int NBLK>
__host__ __device__ constexpr int trsm_npairs() { return NBLK * (NBLK - 1) / 2; }

// p-th (source, target) block pair: forward sweep b = 0.., b' = b+1..;
// backward sweep b = NBLK-1..1, b' = 0..b-1.
template <int NBLK>
__host__ __device__ constexpr int trsm_pair(int p, bool fwd, bool want_src) {
    int q = 0;
    for (int s = 0; s < NBLK; ++s) {
        const int b = fwd ? s : NBLK - 1 - s;
        const int lo = fwd ? b + 1 : 0, hi = fwd ? NBLK : b;
        for (int bp = lo; bp < hi; ++bp) {
            if (q == p) return want_src ? b : bp;
            ++q;
        }
    }
    return 0;
}

// x_bp -= T_{bp,b} x_b (the operand already negated)
template <int NBLK, int NT16, int B, int BP, class CT, class V4>
__device__ __forceinline__ void trsmw_update(V4 (&x)[NBLK][2][NT16], const CT (&o)[2][8]) {
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int nt = 0; nt < NT16; ++nt)
                x[BP][tr][nt] = mfma4(o[tr][kk], x[B][kk >> 2][nt][kk & 3], x[BP][tr][nt]);
}

// ------------------------------------------------------------------ triangular solves, operands shared in LDS
//
// A workgroup of WPB waves covers WPB consecutive slabs of one chunk (the
// register layout above) and the 32 x 32 factor blocks go through LDS once
// per workgroup instead of once per wave: the blocks of the whole sequence (forward block
// pairs, inverses of the diagonal blocks of L, backward pairs, inverses of
// the diagonal blocks of U) stream through a ring of four LDS slots, each
// thread loading one 32-byte piece two blocks ahead, with one barrier per
// block.  A staged block is stored in operand order: lane l's 16 left
// operands (two row tiles x eight k) are contiguous, lanes 80 bytes apart,
// so the reads are free of bank conflicts.
constexpr int TS_LANE = 10;                  // doubles per lane and row tile in a staged block
constexpr int TS_BLOCK = 2 * 64 * TS_LANE;   // doubles per staged block
constexpr int TS_RING = 4;

template <int NBLK>
__host__ __device__ constexpr int trsm_nseq() { return 2 * (trsm_npairs<NBLK>() + NBLK); }

// Element e of the block sequence: kind 0 forward pair, 1 diagonal of L,
// 2 backward pair, 3 diagonal of U; source block (b) and target block (bp).
template <int NBLK>
__host__ __device__ constexpr int tseq_kind(int e) {
    constexpr int NP = trsm_npairs<NBLK>();
    return e < NP ? 0 : e < NP + NBLK ? 1 : e < 2 * NP + NBLK ? 2 : 3;
}
template <int NBLK>
__host__ __device__ constexpr int tseq_b(int e) {
    constexpr int NP = trsm_npairs<NBLK>();
    const int k = tseq_kind<NBLK>(e);
    return k == 0 ? trsm_pair<NBLK>(e, true, true)
         : k == 1 ? e - NP
         : k == 2 ? trsm_pair<NBLK>(e - NP - NBLK, false, true)
                  : e - 2 * NP - NBLK;
}
template <int NBLK>
__host__ __device__ constexpr int tseq_bp(int e) {
    constexpr int NP = trsm_npairs<NBLK>();
    const int k = tseq_kind<NBLK>(e);
    return k == 0 ? trsm_pair<NBLK>(e, true, false)
         : k == 2 ? trsm_pair<NBLK>(e - NP - NBLK, false, false)
                  : tseq_b<NBLK>(e);
}

// This thread's piece of sequence element e: PC = 4 or 2 consecutive doubles
// of one block row, loaded as they are.  Every load is made, from a clamped
// address where the piece reaches past the matrix; the bits of `valid` say
// which values are inside.  The sign change of the pairs and the zeros
// outside are applied when the piece is staged, two elements later: no
// divergent branch and no use of the loaded values follows the loads, so
// the loads of later elements stay in flight while earlier pieces are
// staged.
template <int NBLK, int PC>
__device__ __forceinline__ double4 tseq_load(int e, const double* __restrict__ lu, const double* __restrict__ di,
                                             int M, int nblk, int tid, int& valid) {
    const int kind = tseq_kind<NBLK>(e), b = tseq_b<NBLK>(e), bp = tseq_bp<NBLK>(e);
    constexpr int PR = DB / PC;   // pieces per block row
    // the thread index made opaque here: each element's address is formed
    // where it is loaded instead of all of them up front (registers)
    int to = tid;
    __asm__ volatile("" : "+v"(to));
    const int r = to / PR, c4 = (to % PR) * PC;
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    valid = 0;
    if (kind == 0 || kind == 2) {
        const int row = bp * DB + r, col = b * DB + c4;
        const int rs = row < M ? row : 0;
#pragma unroll
        for (int u = 0; u < PC; ++u) {
            q[u] = lu[(uint32_t)(rs * M + min(col + u, M - 1))];
            valid |= (row < M && col + u < M) ? 1 << u : 0;
        }
    } else {
        const int bs = b < nblk ? b : 0;
        const double* src = di + (size_t)bs * DI_STRIDE + (kind == 3 ? DB * DB : 0) + r * DB + c4;
        if (PC == 4) {
            const double4 v = *(const double4*)src;
            q[0] = v.x; q[1] = v.y; q[2] = v.z; q[3] = v.w;
        } else {
            const double2 h = *(const double2*)src;
            q[0] = h.x; q[1] = h.y;
        }
        valid = b < nblk ? 15 : 0;
    }
    return make_double4(q[0], q[1], q[2], q[3]);
}

// Store a piece of sequence element e in operand order (negated for pairs,
// zeros outside the matrix), rounded to the product type CT: block row r
// (held in lane group g = r >> 3, register v = r & 3 of row tile
// tr = (r >> 2) & 1) is the MFMA output row i16 that register v of lane group
// g holds; column c = 8 g + kk.
template <int NBLK, int PC, class CT = double>
__device__ __forceinline__ void tseq_stage(int e, CT* slot, int tid, double4 v, int valid) {
    constexpr int PR = DB / PC;
    const int kind = tseq_kind<NBLK>(e);
    const double sg = (kind == 0 || kind == 2) ? -1.0 : 1.0;
    const double x0 = (valid & 1) ? sg * v.x : 0.0, x1 = (valid & 2) ? sg * v.y : 0.0;
    const double x2 = (valid & 4) ? sg * v.z : 0.0, x3 = (valid & 8) ? sg * v.w : 0.0;
    const int r = tid / PR, c4 = (tid % PR) * PC;
    const int tr = (r >> 2) & 1, i16 = mfma_row<CT>((r >> 3) << 4, r & 3);
    const int g = c4 >> 3, kk = c4 & 7;
    CT* d = slot + (tr * 64 + g * 16 + i16) * TS_LANE + kk;
    if constexpr (sizeof(CT) == 8) {
        *(double2*)d = make_double2(x0, x1);
        if (PC == 4) *(double2*)(d + 2) = make_double2(x2, x3);
    } else {
        *(float2*)d = make_float2((float)x0, (float)x1);
        if (PC == 4) *(float2*)(d + 2) = make_float2((float)x2, (float)x3);
    }
}

template <int NBLK, int NT16, int E, class CT = double>
__device__ __forceinline__ void tseq_apply(typename Acc4<CT>::type (&x)[NBLK][2][NT16], const CT* slot, int lane) {
    typedef typename Acc4<CT>::type V4;
    constexpr int kind = tseq_kind<NBLK>(E), B = tseq_b<NBLK>(E), BP = tseq_bp<NBLK>(E);
    CT o[2][8];
#pragma unroll
    for (int tr = 0; tr < 2; ++tr) {
        const CT* src = slot + (tr * 64 + lane) * TS_LANE;
        if constexpr (sizeof(CT) == 8) {
            const double2 a0 = *(const double2*)src, a1 = *(const double2*)(src + 2);
            const double2 a2 = *(const double2*)(src + 4), a3 = *(const double2*)(src + 6);
            o[tr][0] = a0.x; o[tr][1] = a0.y; o[tr][2] = a1.x; o[tr][3] = a1.y;
            o[tr][4] = a2.x; o[tr][5] = a2.y; o[tr][6] = a3.x; o[tr][7] = a3.y;
        } else {
            const float2 a0 = *(const float2*)src, a1 = *(const float2*)(src + 2);
            const float2 a2 = *(const float2*)(src + 4), a3 = *(const float2*)(src + 6);
            o[tr][0] = a0.x; o[tr][1] = a0.y; o[tr][2] = a1.x; o[tr][3] = a1.y;
            o[tr][4] = a2.x; o[tr][5] = a2.y; o[tr][6] = a3.x; o[tr][7] = a3.y;
        }
    }
    if constexpr (kind == 0 || kind == 2) {
        trsmw_update<NBLK, NT16, B, BP>(x, o);
    } else {
        V4 nw[2][NT16];
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int nt = 0; nt < NT16; ++nt) nw[tr][nt] = (V4){0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int tr = 0; tr < 2; ++tr)
#pragma unroll
                for (int nt = 0; nt < NT16; ++nt) nw[tr][nt] = mfma4(o[tr][kk], x[B][kk >> 2][nt][kk & 3], nw[tr][nt]);
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int nt = 0; nt < NT16; ++nt) x[B][tr][nt] = nw[tr][nt];
    }
}

// Sequence element E: stage E+1 (loaded two elements ago), start loading
// E+3, apply E, barrier.  p0/p1 (validity m0/m1) hold the pieces of E+1 and
// E+2 on entry.
template <int NBLK, int NT16, int PC, int E, class CT = double>
__device__ __forceinline__ void tseq_run(typename Acc4<CT>::type (&x)[NBLK][2][NT16], CT* ring,
                                         const double* __restrict__ lu, const double* __restrict__ di, int M, int nblk,
                                         int tid, int lane, double4& p0, int m0, double4& p1, int m1) {
    constexpr int NS = trsm_nseq<NBLK>();
    if constexpr (E < NS) {
        if constexpr (E + 1 < NS) tseq_stage<NBLK, PC, CT>(E + 1, ring + ((E + 1) % TS_RING) * TS_BLOCK, tid, p0, m0);
        double4 p2 = {0.0, 0.0, 0.0, 0.0};
        int m2 = 0;
        if constexpr (E + 3 < NS) p2 = tseq_load<NBLK, PC>(E + 3, lu, di, M, nblk, tid, m2);
        tseq_apply<NBLK, NT16, E, CT>(x, ring + (E % TS_RING) * TS_BLOCK, lane);
        __syncthreads();
        tseq_run<NBLK, NT16, PC, E + 1, CT>(x, ring, lu, di, M, nblk, tid, lane, p1, m1, p2, m2);
    }
}

// The same two elements per barrier (the number of elements is even):
// elements E, E+1 were staged before the barrier that ends the previous
// pair; stage E+2, E+3 (loaded two pairs ago), start loading E+6, E+7,
// apply E and E+1, barrier.  q0..q3 hold the pieces of E+2 .. E+5 on entry.
// The four ring slots of E .. E+3 are distinct.
template <int NBLK, int NT16, int PC, int E, class CT = double>
__device__ __forceinline__ void tseq_run2(typename Acc4<CT>::type (&x)[NBLK][2][NT16], CT* ring,
                                          const double* __restrict__ lu, const double* __restrict__ di, int M,
                                          int nblk, int tid, int lane, double4& q0, int n0, double4& q1, int n1,
                                          double4& q2, int n2, double4& q3, int n3) {
    constexpr int NS = trsm_nseq<NBLK>();
    static_assert(NS % 2 == 0, "pairs of sequence elements");
    if constexpr (E < NS) {
        if constexpr (E + 2 < NS) {
            tseq_stage<NBLK, PC, CT>(E + 2, ring + ((E + 2) % TS_RING) * TS_BLOCK, tid, q0, n0);
            tseq_stage<NBLK, PC, CT>(E + 3, ring + ((E + 3) % TS_RING) * TS_BLOCK, tid, q1, n1);
        }
        double4 q4 = {0.0, 0.0, 0.0, 0.0}, q5 = {0.0, 0.0, 0.0, 0.0};
        int n4 = 0, n5 = 0;
        if constexpr (E + 6 < NS) {
            q4 = tseq_load<NBLK, PC>(E + 6, lu, di, M, nblk, tid, n4);
            q5 = tseq_load<NBLK, PC>(E + 7, lu, di, M, nblk, tid, n5);
        }
        tseq_apply<NBLK, NT16, E, CT>(x, ring + (E % TS_RING) * TS_BLOCK, lane);
        __builtin_amdgcn_sched_barrier(0);   // one element's operands at a time (registers)
        tseq_apply<NBLK, NT16, E + 1, CT>(x, ring + ((E + 1) % TS_RING) * TS_BLOCK, lane);
        __syncthreads();
        tseq_run2<NBLK, NT16, PC, E + 2, CT>(x, ring, lu, di, M, nblk, tid, lane, q2, n2, q3, n3, q4, n4, q5, n5);
    }
}

// RHS: the right-hand-side sweep's X_i (R columns, in place) instead of
// W_i = [C_i | -B_i Y_{i-1}].  CT: product type (float: FP32 MFMA with FP32
// accumulation on the FP64 factors and right-hand side, for the
// reduced-precision factor; results stored in FP64).  WPE: waves per SIMD
// the register allocation must admit (2: at most 256 VGPRs, so that two
// four-wave workgroups share a CU and one's barriers are covered by the
// other's products).
template <int NBLK, int NT16, int WPB, bool RHS = false, class CT = double, int WPE = 1>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(WPE))) void k_getrs_s(const KArgs ka,
                                                                                                  int nslab, int wpc) {
    typedef typename Acc4<CT>::type V4;
    __shared__ CT ring[TS_RING * TS_BLOCK];
    const Level& L = ka.L;
    const int M = L.M;
    const int lid = xcd_logical_id(blockIdx.x, gridDim.x);
    const int k = ka.c0 + lid / wpc, wgc = lid % wpc;
    const int r = chunk_first(L, k), e = chunk_last(L, k), t = ka.step;
    if (t > e - r) return;
    const int i = r + t;
    constexpr int SW = 16 * NT16;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, j = lane & 15;
    // solved columns: E_i [0, e_hi) and Y_i [M, y_hi) of W_i, or [0, R) of X_i
    const int e_hi = RHS ? ka.R : (i != L.N - 1) ? M : 0;
    const int y_hi = RHS ? 0 : (k > 0) ? 2 * M : M;
    const int g0 = wgc * WPB * SW, g1 = min(g0 + WPB * SW, nslab * SW);
    if (!(g0 < e_hi || (g0 < y_hi && g1 > M))) return;   // nothing to solve in this workgroup
    const int slab = wgc * WPB + w;
    const int c0 = slab * SW;
    const int nblk = (M + DB - 1) / DB;
    const double* lu = L.LU + (size_t)i * M * M;
    const double* di = L.DI + (size_t)i * nblk * DI_STRIDE;
    const int* perm = L.perm + (size_t)i * M;
    double* X = RHS ? ka.X + (size_t)i * M * ka.R : L.W + (size_t)i * M * 2 * M;
    const int ld = RHS ? ka.R : 2 * M;
    // first blocks of the sequence in flight before the right-hand side is read
    constexpr int PC = 1024 / (64 * WPB);   // doubles of a staged block per thread
    int m0, m1, m2, m3, m4, m5;
    double4 p0 = tseq_load<NBLK, PC>(0, lu, di, M, nblk, tid, m0);
    double4 p1 = tseq_load<NBLK, PC>(1, lu, di, M, nblk, tid, m1);
    double4 p2 = tseq_load<NBLK, PC>(2, lu, di, M, nblk, tid, m2);
    double4 p3 = tseq_load<NBLK, PC>(3, lu, di, M, nblk, tid, m3);
    double4 p4 = tseq_load<NBLK, PC>(4, lu, di, M, nblk, tid, m4);
    double4 p5 = tseq_load<NBLK, PC>(5, lu, di, M, nblk, tid, m5);
    // the right-hand side from the pivot rows (perm holds valid rows), every
    // load unconditional from a clamped row and column; zeros outside after
    // all loads are out.  The E half of W_i starts as C_i and is read from C
    // (the forward product does not copy it for this kernel); the solution
    // goes to W_i.
    const double* Ci = RHS ? X : L.C + (size_t)i * M * M;
    // at a chunk's first row the Y half starts as B_i, read from B itself (no
    // forward product runs at that step)
    const bool seed = !RHS && t == 0;
    const double* Bi = L.B + (size_t)i * M * M;
    V4 x[NBLK][2][NT16];
#pragma unroll
    for (int b = 0; b < NBLK; ++b)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr) {
            int prw[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) prw[v] = perm[min(b * DB + 8 * g + 4 * tr + v, M - 1)];
#pragma unroll
            for (int nt = 0; nt < NT16; ++nt) {
                const int col = c0 + 16 * nt + j;
                const bool cv = col < e_hi || (col >= M && col < y_hi);
                const bool fromC = !RHS && cv && col < M;
                const bool fromB = seed && cv && col >= M;
                const double* src = fromC ? Ci : fromB ? Bi : X;
                const int lds = (fromC || fromB) ? M : ld;
                const int cs = !cv ? 0 : fromB ? col - M : col;
#pragma unroll
                for (int v = 0; v < 4; ++v) x[b][tr][nt][v] = (CT)src[(uint32_t)(prw[v] * lds + cs)];
            }
        }
#pragma unroll
    for (int b = 0; b < NBLK; ++b)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int nt = 0; nt < NT16; ++nt) {
                const int col = c0 + 16 * nt + j;
                const bool cv = col < e_hi || (col >= M && col < y_hi);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = b * DB + 8 * g + 4 * tr + v;
                    x[b][tr][nt][v] = (cv && row < M) ? x[b][tr][nt][v] : (CT)0;
                }
            }
    tseq_stage<NBLK, PC, CT>(0, ring, tid, p0, m0);
    tseq_stage<NBLK, PC, CT>(1, ring + TS_BLOCK, tid, p1, m1);
    __syncthreads();
    tseq_run2<NBLK, NT16, PC, 0, CT>(x, ring, lu, di, M, nblk, tid, lane, p2, m2, p3, m3, p4, m4, p5, m5);
    // at a chunk's last row the spikes start the backward sweep as they
    // are: Z_e = [Z_L | Z_R] = [Y_e | E_e], written here as well (the
    // backward sweep runs no step for that row)
    const bool zlast = !RHS && L.P > 1 && i == e;
    double* Ze = L.Z + (size_t)i * M * 2 * M;
#pragma unroll
    for (int b = 0; b < NBLK; ++b)
#pragma unroll
        for (int tr = 0; tr < 2; ++tr)
#pragma unroll
            for (int nt = 0; nt < NT16; ++nt) {
                const int col = c0 + 16 * nt + j;
                const bool cv = col < e_hi || (col >= M && col < y_hi);
                const int zc = col < M ? col + M : col - M;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = b * DB + 8 * g + 4 * tr + v;
                    if (cv && row < M && zlast) Ze[(uint32_t)(row * 2 * M + zc)] = (double)x[b][tr][nt][v];
                    if (cv && row < M) X[(uint32_t)(row * ld + col)] = (double)x[b][tr][nt][v];
                }
            }
}

// ------------------------------------------------------------------ right-hand-side sweeps
//
// One workgroup per (chunk, group of RB columns) runs the chunk's whole
// right-hand-side sweep (the F part of Eq. e231 by the Thomas algorithm of
// Sec. 3 with LU factors):
//   forward   y_i = U_i^{-1} L_i^{-1} P_i (F_i - B_i y_{i-1})
//   backward  z_i = y_i - E_i z_{i+1}   (z_last = y_last)
// The working block (M x RB) lives in LDS; B_i and E_i stream through LDS in
// 32-column panels read row-contiguously; the triangular solves go by 32-row
// blocks with the inverted diagonal blocks and the off-diagonal panel read
// straight from the LU factors.  The solution is written to X (rows of the
// chunk), which may alias F.
template <int RB, int KC>
__device__ __forceinline__ void lds_gemv_sub(const double* __restrict__ Mat, int ld, int M, const double* v, double* t,
                                             double* st) {
    // t (M x RB, LDS) -= Mat (M x M, row-major, global) * v (M x RB, LDS); the
    // next KC-column panel is loaded into registers while the current one is used
    const int tid = threadIdx.x;
    constexpr int SP = KC + 1;
    constexpr int PER = (BTD_MAX_M * KC + 255) / 256 > 32 ? 32 : (BTD_MAX_M * KC + 255) / 256;
    double nx[PER];
    auto load_panel = [&](int kc) {
        const int kw = min(KC, M - kc);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = tid + u * 256, rr = idx / KC, cc = idx - rr * KC;
            nx[u] = (rr < M && cc < kw) ? Mat[(size_t)rr * ld + kc + cc] : 0.0;
        }
    };
    load_panel(0);
    for (int kc = 0; kc < M; kc += KC) {
        const int kw = min(KC, M - kc);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int idx = tid + u * 256, rr = idx / KC, cc = idx - rr * KC;
            if (rr < M) st[rr * SP + cc] = nx[u];
        }
        __syncthreads();
        if (kc + KC < M) load_panel(kc + KC);
        for (int rr = tid; rr < M; rr += 256) {
            double acc[RB];
#pragma unroll
            for (int c = 0; c < RB; ++c) acc[c] = 0.0;
#pragma unroll 8
            for (int cc = 0; cc < KC; ++cc) {
                if (cc < kw) {
                    const double m = st[rr * SP + cc];
#pragma unroll
                    for (int c = 0; c < RB; ++c) acc[c] += m * v[(kc + cc) * RB + c];
                }
            }
#pragma unroll
            for (int c = 0; c < RB; ++c) t[rr * RB + c] -= acc[c];
        }
    }
    __syncthreads();
}

template <int RB>
__device__ __forceinline__ void lds_lu_solve(const double* __restrict__ lu, const double* __restrict__ di, int M,
                                             double* t, double* t2) {
    // t := U^{-1} L^{-1} t (rows already permuted) with the scaled
    // off-diagonal blocks: each sweep step updates the other rows with the
    // unsolved block (one barrier), then all diagonal blocks are solved at
    // once.  t2 is scratch; the result ends in t.
    const int tid = threadIdx.x;
    const int nblk = (M + DB - 1) / DB;
    for (int dir = 0; dir < 2; ++dir) {
        for (int step = 0; step < nblk; ++step) {
            const int bb = dir == 0 ? step : nblk - 1 - step;
            const int b0 = bb * DB, bs = min(DB, M - b0);
            const int lo = dir == 0 ? b0 + bs : 0, hi = dir == 0 ? M : b0;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int rr = lo + tid + q * 256;
                if (rr < hi) {
                    double seg[DB];
#pragma unroll
                    for (int j = 0; j < DB; ++j) seg[j] = j < bs ? lu[(size_t)rr * M + b0 + j] : 0.0;
                    double acc[RB];
#pragma unroll
                    for (int c = 0; c < RB; ++c) acc[c] = 0.0;
#pragma unroll
                    for (int j = 0; j < DB; ++j) {
                        if (j < bs) {
#pragma unroll
                            for (int c = 0; c < RB; ++c) acc[c] += seg[j] * t[(b0 + j) * RB + c];
                        }
                    }
#pragma unroll
                    for (int c = 0; c < RB; ++c) t[rr * RB + c] -= acc[c];
                }
            }
            __syncthreads();
        }
        // all diagonal blocks at once: t2 = inv(T_bb) t_b
        for (int rr = tid; rr < M; rr += 256) {
            const int bb = rr / DB, b0 = bb * DB, bs = min(DB, M - b0);
            const double* inv = di + (size_t)bb * DI_STRIDE + (dir == 0 ? 0 : DB * DB) + (size_t)(rr - b0) * DB;
            double iv[DB];
#pragma unroll
            for (int j = 0; j < DB; ++j) iv[j] = inv[j];
            double acc[RB];
#pragma unroll
            for (int c = 0; c < RB; ++c) acc[c] = 0.0;
#pragma unroll
            for (int j = 0; j < DB; ++j) {
                if (j < bs) {
#pragma unroll
                    for (int c = 0; c < RB; ++c) acc[c] += iv[j] * t[(b0 + j) * RB + c];
                }
            }
#pragma unroll
            for (int c = 0; c < RB; ++c) t2[rr * RB + c] = acc[c];
        }
        __syncthreads();
        double* sw = t;
        t = t2;
        t2 = sw;
    }
}

template <int RB, int KC>
__global__ __launch_bounds__(256) void k_chunk_solve(const KArgs ka) {
    const Level& L = ka.L;
    const int k = blockIdx.x, c0 = blockIdx.y * RB, R = ka.R, M = L.M;
    if (c0 >= R) return;
    const int nc = min(RB, R - c0);
    const int r0 = chunk_first(L, k), e = chunk_last(L, k);
    const int nblk = (M + DB - 1) / DB;
    const int tid = threadIdx.x;
    extern __shared__ double sm[];
    double* ya = sm;                       // [M][RB] previous row's block
    double* tb = ya + (size_t)M * RB;      // [M][RB] current block
    double* tp = tb + (size_t)M * RB;      // [M][RB] permutation buffer
    double* tmp = tp + (size_t)M * RB;     // [DB][RB]
    double* ib = tmp + DB * RB;            // [DB][DB] inverted diagonal block
    double* st = ib + DB * DB;             // [M][KC+1] staging panel
    const size_t MM = (size_t)M * M, MR = (size_t)M * R;
    // forward sweep
    for (int i = r0; i <= e; ++i) {
        copy_batched<8>(
            M * RB,
            [&](int idx) {
                const int rr = idx / RB, c = idx - rr * RB;
                return c < nc ? ka.F[i * MR + (size_t)rr * R + c0 + c] : 0.0;
            },
            [&](int idx, double v) { tb[idx] = v; });
        __syncthreads();
        PHASE_MARK(g0);
        if (i > r0) lds_gemv_sub<RB, KC>(L.B + i * MM, M, M, ya, tb, st);
        PHASE_MARK(g1);
        PHASE_ADD(8, g0, g1);
        const int* perm = L.perm + (size_t)i * M;
        for (int idx = tid; idx < M * RB; idx += 256) {
            const int rr = idx / RB, c = idx - rr * RB;
            tp[idx] = tb[perm[rr] * RB + c];
        }
        __syncthreads();
        PHASE_MARK(l0);
        lds_lu_solve<RB>(L.LU + i * MM, L.DI + (size_t)i * nblk * DI_STRIDE, M, tp, tb);
        PHASE_MARK(l1);
        PHASE_ADD(9, l0, l1);
        for (int idx = tid; idx < M * RB; idx += 256) {
            const int rr = idx / RB, c = idx - rr * RB;
            ya[idx] = tp[idx];
            if (c < nc) ka.X[i * MR + (size_t)rr * R + c0 + c] = tp[idx];
        }
        __syncthreads();
    }
    // backward sweep: ya holds z of the row below
    for (int i = e - 1; i >= r0; --i) {
        copy_batched<8>(
            M * RB,
            [&](int idx) {
                const int rr = idx / RB, c = idx - rr * RB;
                return c < nc ? ka.X[i * MR + (size_t)rr * R + c0 + c] : 0.0;
            },
            [&](int idx, double v) { tb[idx] = v; });
        __syncthreads();
        lds_gemv_sub<RB, KC>(L.W + i * MM * 2, 2 * M, M, ya, tb, st);
        for (int idx = tid; idx < M * RB; idx += 256) {
            const int rr = idx / RB, c = idx - rr * RB;
            ya[idx] = tb[idx];
            if (c < nc) ka.X[i * MR + (size_t)rr * R + c0 + c] = tb[idx];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ right-hand-side sweep, one column
//
// The sweep of k_chunk_solve for R = 1 and M a multiple of 64, shaped to
// run beside the factorization's product kernels on the same CUs (at most
// 128 VGPRs per lane and a few KiB of LDS, where k_chunk_solve's register
// file and LDS leave no room for another workgroup).  One workgroup per
// chunk; every step is a set of products of matrix rows with a vector in
// LDS, 16 lanes per row (four rows per wave instruction) and a DPP sum over
// the 16 lanes:
//   forward, row i:  t = P_i (F_i - B_i y_{i-1})   (rows of B_i, F_i taken in pivot order)
//                    t := L_i^{-1} t   by 32-row blocks: the rows below block b subtract the
//                                      product of their (scaled) segment of block b with t_b,
//                                      then every block takes the inverse of its diagonal
//                                      block of L
//                    y_i = U_i^{-1} t  the same upwards with the blocks of U
//   backward, row i: z_i = y_i - E_i z_{i+1}
// (the F part of Eq. e231 by the Thomas algorithm of Sec. 3 with the LU
// factors).  The kernel is bound by load latency (one workgroup per chunk),
// so its loads run two batches ahead: a batch's products are formed, the
// batch after next is loaded into the same registers, then the sums are
// reduced and written; the factor loads do not depend on the vector, so
// they cross the barriers between steps.  Loads come from clamped
// addresses, unconditionally.

// Sum over each 16-lane row; every lane of the row holds the row's sum.
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return v;
}

constexpr int RS_BATCH = 8;   // passes of 16 rows per batch of the triangular solve

// Streaming loads of the factors (non-temporal: the sweep reads each value
// once, and runs beside product kernels whose operands live in L2).
typedef double v2d __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream2(const double* p) {
    const v2d v = __builtin_nontemporal_load((const v2d*)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ double4 ld_stream4(const double* p) {
    const v4d v = __builtin_nontemporal_load((const v4d*)p);
    return make_double4(v.x, v.y, v.z, v.w);
}

// One batch of the triangular solve of a row: kind 0 a step of L (block bb,
// the rows below it), 1 the diagonal blocks of L, 2 a step of U (block bb,
// the rows above it), 3 the diagonal blocks of U; passes p0 .. p0 + 7 of np;
// `last`: the last batch of its step (a barrier follows).
struct RsUnit {
    int kind, bb, p0, np;
    bool last;
};

template <int NBLK>
struct RsPlan {
    static constexpr int nb(int np) { return (np + RS_BATCH - 1) / RS_BATCH; }
    static constexpr int count() {
        int n = 0;
        for (int bb = 0; bb + 1 < NBLK; ++bb) n += nb(2 * (NBLK - 1 - bb));
        n += nb(2 * NBLK);
        for (int bb = NBLK - 1; bb > 0; --bb) n += nb(2 * bb);
        return n + nb(2 * NBLK);
    }
    static constexpr RsUnit unit(int want) {
        int n = 0;
        for (int ph = 0; ph < 4; ++ph) {
            const int steps = (ph == 1 || ph == 3) ? 1 : NBLK - 1;
            for (int s = 0; s < steps; ++s) {
                const int bb = ph == 0 ? s : ph == 2 ? NBLK - 1 - s : 0;
                const int np = ph == 0 ? 2 * (NBLK - 1 - bb) : ph == 2 ? 2 * bb : 2 * NBLK;
                for (int q = 0; q < nb(np); ++q, ++n)
                    if (n == want) return RsUnit{ph, bb, q * RS_BATCH, np, q + 1 == nb(np)};
            }
        }
        return RsUnit{-1, 0, 0, 0, false};
    }
};

// Row of pass p of a unit for this lane's row group.
__device__ __forceinline__ int rs_row(const RsUnit& u, int p, int w, int g) {
    const int lo = u.kind == 0 ? DB * (u.bb + 1) : 0;
    return lo + 16 * p + 4 * w + g;
}

template <int NBLK, int N>
__device__ __forceinline__ void rs_load(double2 (&v)[RS_BATCH], const double* __restrict__ lu,
                                        const double* __restrict__ di, int lane, int w) {
    constexpr int M = NBLK * DB;
    constexpr RsUnit u = RsPlan<NBLK>::unit(N);
    if constexpr (u.kind >= 0) {
        // the lane's indices made opaque per batch: addresses are formed at
        // the loads instead of for every batch up front (registers)
        int lo = lane, wo = w;
        __asm__ volatile("" : "+v"(lo), "+v"(wo));
        const int j = lo & 15, g = lo >> 4;
        w = wo;
#pragma unroll
        for (int pb = 0; pb < RS_BATCH; ++pb) {
            const int r = rs_row(u, min(u.p0 + pb, u.np - 1), w, g);
            if constexpr (u.kind == 0 || u.kind == 2)
                v[pb] = ld_stream2(lu + (size_t)r * M + DB * u.bb + 2 * j);
            else
                v[pb] = ld_stream2(di + (size_t)(r >> 5) * DI_STRIDE + (u.kind == 3 ? DB * DB : 0) + (r & 31) * DB +
                                   2 * j);
        }
    }
}

// Unit N from va; unit N + 2 is loaded into va once its products are
// formed; then N + 1 from vb.  The vector is in ta (L steps, the diagonal
// of L reads ta and writes tc; U steps in tc, the diagonal of U reads tc
// and writes ta and the row of X).
template <int NBLK, int N>
__device__ __forceinline__ void rs_run(double2 (&va)[RS_BATCH], double2 (&vb)[RS_BATCH], const double* __restrict__ lu,
                                       const double* __restrict__ di, double* ta, double* tc, double* xg, int lane,
                                       int w) {
    constexpr int NU = RsPlan<NBLK>::count();
    if constexpr (N < NU) {
        constexpr RsUnit u = RsPlan<NBLK>::unit(N);
        int lo = lane, wo = w;
        __asm__ volatile("" : "+v"(lo), "+v"(wo));
        const int j = lo & 15, g = lo >> 4;
        double part[RS_BATCH];
        if constexpr (u.kind == 0 || u.kind == 2) {
            const double* t = u.kind == 0 ? ta : tc;
            const double u0 = t[DB * u.bb + 2 * j], u1 = t[DB * u.bb + 2 * j + 1];
#pragma unroll
            for (int pb = 0; pb < RS_BATCH; ++pb) part[pb] = fma(va[pb].x, u0, va[pb].y * u1);
        } else {
            const double* t = u.kind == 1 ? ta : tc;
#pragma unroll
            for (int pb = 0; pb < RS_BATCH; ++pb) {
                const int b0 = rs_row(u, u.p0 + pb, wo, g) & ~31;
                part[pb] = fma(va[pb].x, t[b0 + 2 * j], va[pb].y * t[b0 + 2 * j + 1]);
            }
        }
        rs_load<NBLK, N + 2>(va, lu, di, lane, w);
#pragma unroll
        for (int pb = 0; pb < RS_BATCH; ++pb) {
            const double a = row16_sum(part[pb]);
            if (u.p0 + pb < u.np && j == 0) {
                const int r = rs_row(u, u.p0 + pb, wo, g);
                if constexpr (u.kind == 0) ta[r] -= a;
                else if constexpr (u.kind == 2) tc[r] -= a;
                else if constexpr (u.kind == 1) tc[r] = a;
                else {
                    ta[r] = a;
                    xg[r] = a;
                }
            }
        }
        if constexpr (u.last) __syncthreads();
        rs_run<NBLK, N + 1>(vb, va, lu, di, ta, tc, xg, lane, w);
    }
}

// Rows q = 16 p + 4 w + g (p < M / 16) of outl (LDS) and outg (global, optional):
// out[q] = base[s] - Mx[s, :] y with s = pm[q] (PERM) or q, Mx row-major with
// leading dimension ld (no product unless HASM), y in LDS; lane j covers the
// columns 4 j + 64 c, c < NPC.  Up to M = 256 two passes are in flight (the
// pass after next loaded once a pass's products are formed).
template <int NPC, bool HASM, bool PERM>
__device__ __forceinline__ void rs_gemv(const double* __restrict__ Mx, int ld, const int* pm, const double* base,
                                        const double* y, double* outl, double* outg, int lane, int w) {
    constexpr int M = 64 * NPC, NP = M / 16;
    constexpr int AHEAD = NPC <= 4 ? 2 : 1;
    const int j = lane & 15, g = lane >> 4;
    double4 v[AHEAD][HASM ? NPC : 1];
    double bs[AHEAD];
    auto load = [&](int p, double4 (&d)[HASM ? NPC : 1], double& b) {
        const int q = 16 * min(p, NP - 1) + 4 * w + g;
        const int sr = PERM ? pm[q] : q;
        b = base[sr];
        if constexpr (HASM) {
#pragma unroll
            for (int c = 0; c < NPC; ++c) d[c] = ld_stream4(Mx + (size_t)sr * ld + 4 * j + 64 * c);
        }
    };
#pragma unroll
    for (int k = 0; k < AHEAD; ++k) load(k, v[k], bs[k]);
    for (int p0 = 0; p0 < NP; p0 += AHEAD) {
#pragma unroll
        for (int k = 0; k < AHEAD; ++k) {
            const int p = p0 + k;
            double a = 0.0;
            if constexpr (HASM) {
#pragma unroll
                for (int c = 0; c < NPC; ++c) {
                    const double4 yv = *(const double4*)(y + 4 * j + 64 * c);
                    a = fma(v[k][c].x, yv.x, a);
                    a = fma(v[k][c].y, yv.y, a);
                    a = fma(v[k][c].z, yv.z, a);
                    a = fma(v[k][c].w, yv.w, a);
                }
            }
            const double b = bs[k];
            load(p + AHEAD, v[k], bs[k]);
            a = row16_sum(a);
            if (j == 0) {
                const int q = 16 * p + 4 * w + g;
                const double r = b - a;
                outl[q] = r;
                if (outg) outg[q] = r;
            }
        }
    }
}

// Forward row i of a chunk (first row r0): pm holds P_i, ya y_{i-1}; the
// solution goes to tb and X_i.
template <int NPC>
__device__ __forceinline__ void rs_forward_row(const KArgs& ka, int i, int r0, const int* pm, const double* ya,
                                               double* tb, double* t2, int lane, int w) {
    constexpr int M = 64 * NPC, NBLK = M / DB;
    const Level& L = ka.L;
    const size_t MM = (size_t)M * M;
    const double* LUi = L.LU + i * MM;
    const double* DIi = L.DI + (size_t)i * NBLK * DI_STRIDE;
    if (i > r0) rs_gemv<NPC, true, true>(L.B + i * MM, M, pm, ka.F + (size_t)i * M, ya, tb, nullptr, lane, w);
    else rs_gemv<NPC, false, true>(nullptr, M, pm, ka.F + (size_t)i * M, ya, tb, nullptr, lane, w);
    double2 va[RS_BATCH], vb[RS_BATCH];
    rs_load<NBLK, 0>(va, LUi, DIi, lane, w);
    rs_load<NBLK, 1>(vb, LUi, DIi, lane, w);
    __syncthreads();
    rs_run<NBLK, 0>(va, vb, LUi, DIi, tb, t2, ka.X + (size_t)i * M, lane, w);
}

// Backward rows e-1 .. r0 of a chunk: ya holds z_e on entry.
template <int NPC>
__device__ __forceinline__ void rs_backward(const KArgs& ka, int r0, int e, double* ya, double* tb, int lane, int w) {
    constexpr int M = 64 * NPC;
    const size_t MM = (size_t)M * M;
    for (int i = e - 1; i >= r0; --i) {
        double* Xi = ka.X + (size_t)i * M;
        rs_gemv<NPC, true, false>(ka.L.W + i * MM * 2, 2 * M, nullptr, Xi, ya, tb, Xi, lane, w);
        __syncthreads();
        double* sw = ya; ya = tb; tb = sw;
    }
}

template <int NPC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_rhs_sweep1(const KArgs ka) {
    constexpr int M = 64 * NPC;
    const Level& L = ka.L;
    const int k = blockIdx.x;
    const int r0 = chunk_first(L, k), e = chunk_last(L, k);
    if (e < r0) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    __shared__ double buf[3][M];
    __shared__ int pm[M];
    double* ya = buf[0];   // y of the previous row (z of the next row going back)
    double* tb = buf[1];   // the row being solved
    double* t2 = buf[2];
    constexpr int PU = (M + 255) / 256;
    int pn[PU];            // the next row's permutation, loaded a row ahead
#pragma unroll
    for (int u = 0; u < PU; ++u)
        if (tid + 256 * u < M) pm[tid + 256 * u] = L.perm[(size_t)r0 * M + tid + 256 * u];
    __syncthreads();
    for (int i = r0; i <= e; ++i) {
        const int inext = min(i + 1, e);
#pragma unroll
        for (int u = 0; u < PU; ++u)
            pn[u] = tid + 256 * u < M ? L.perm[(size_t)inext * M + tid + 256 * u] : 0;
        rs_forward_row<NPC>(ka, i, r0, pm, ya, tb, t2, lane, w);
#pragma unroll
        for (int u = 0; u < PU; ++u)
            if (tid + 256 * u < M) pm[tid + 256 * u] = pn[u];
        __syncthreads();
        double* sw = ya; ya = tb; tb = sw;
    }
    rs_backward<NPC>(ka, r0, e, ya, tb, lane, w);
}

// ------------------------------------------------------------------ small utility kernels

__global__ void k_init_status(unsigned long long* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *st = ~0ULL;
}

// Non-finite entries of a right-hand side F [N][M][R] (grid-stride, one
// double per thread and step): each one found reports its (block row,
// column); the smallest key wins in report_status, so the result does not
// depend on the schedule.
__global__ __launch_bounds__(256) void k_check_finite(const double* __restrict__ F, size_t n, int M, int R,
                                                      unsigned long long* st) {
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < n; idx += stride) {
        const double v = F[idx];
        if (!isfinite(v)) report_status(st, 0, (int)(idx / ((size_t)M * R)), (int)(idx % (size_t)R), BTD_ERR_NONFINITE);
    }
}

// X += D over n doubles (the correction of iterative refinement, FP64).
__global__ __launch_bounds__(256) void k_add(double* __restrict__ X, const double* __restrict__ D, size_t n) {
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < n; idx += stride) X[idx] += D[idx];
}

// sep table of a level: written from kernel arguments (no host-to-device copy)
__global__ void k_write_ints(int* dst, int count, IntChunk vals) {
    const int t = threadIdx.x;
    if (t < count) dst[t] = vals.v[t];
}

// ------------------------------------------------------------------ recovery and coupling right-hand side, one column
//
// Both are out = base - [M1 | M2] [v1; v2] over 16 rows per workgroup, with
// M1, M2 two M x M blocks and v1, v2 two vectors of M entries (R = 1):
//   recovery (Eq. endSolution), block row i of chunk k:
//     X_i -= Z_L[i] h^{k-1} + Z_R[i] h^k   (in place; separator rows X_q = h)
//   coupling right-hand side (Eq. e2311), separator q between chunks:
//     Fc_j = F_q - B_q X_{q-1} - C_q X_{q+1}
// M a multiple of 128 and the rows of M1, M2 32-byte aligned: each wave
// takes four whole rows, its lanes covering the 2M columns of [M1 | M2] in
// 32-byte pieces (column kk < M from M1, else column kk - M of M2), the
// matching pieces of [v1; v2] in registers, all four rows' loads in flight
// and a DPP sum per row (an HBM stream of 16 M^2 bytes per item for 4 M^2
// FLOPs).  A block row is split over M / 16 workgroups so that a coupling
// level with few block rows is not one workgroup's stream.
constexpr int RV_ROWS = 16;                        // rows per workgroup
constexpr int RV_MAXP = 2 * BTD_MAX_M / 256;       // 256-column pieces of a 2M row

struct Gemv2 {
    const double* M1;   // row r at M1 + r * ld1
    const double* M2;
    int ld1, ld2;
    const double* v1;   // nullptr: that half is zero
    const double* v2;
    const double* base; // entry r at base[r]
    double* out;        // entry r at out[r] (may alias base)
};

__device__ __forceinline__ void gemv2_rows(const Gemv2& g, int M, int r0, int lane) {
    const int np = 2 * M / 256;
    double hv[RV_MAXP][4];
#pragma unroll
    for (int q = 0; q < RV_MAXP; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int kk = q * 256 + 4 * lane + e;
            const bool isl = kk < M;
            const double* v = isl ? g.v1 : g.v2;
            hv[q][e] = (q < np && v != nullptr) ? v[isl ? kk : kk - M] : 0.0;
        }
    double s[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        s[u] = 0.0;
        const int r = r0 + u;
#pragma unroll
        for (int q = 0; q < RV_MAXP; ++q)
            if (q < np) {
                const int kk = q * 256 + 4 * lane;   // a piece lies in one of the halves (M % 4 == 0)
                const double* src = kk < M ? g.M1 + (size_t)r * g.ld1 + kk : g.M2 + (size_t)r * g.ld2 + (kk - M);
                const double4 zz = *(const double4*)src;
                s[u] = fma(zz.x, hv[q][0], s[u]);
                s[u] = fma(zz.y, hv[q][1], s[u]);
                s[u] = fma(zz.z, hv[q][2], s[u]);
                s[u] = fma(zz.w, hv[q][3], s[u]);
            }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const double tot = wave_sum(s[u]);
        if (lane == 0) g.out[r0 + u] = g.base[r0 + u] - tot;
    }
}

// Recovery: blockIdx.x block row i, blockIdx.y its 16-row slice.
__global__ __launch_bounds__(256) void k_recover_v(const KArgs ka) {
    const Level& L = ka.L;
    const int i = blockIdx.x, M = L.M, P = L.P;
    const int row0 = blockIdx.y * RV_ROWS;
    const size_t MM = (size_t)M * M;
    int lo = 0, hi = P;   // chunk k with sep[k] <= i < sep[k+1]  (sep[0] = -1, sep[P] = N)
    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (L.sep[mid] <= i) lo = mid; else hi = mid; }
    const int k = lo;
    double* Xi = ka.X + (size_t)i * M;
    if (L.sep[k] == i) {   // separator row: X_q = h^k (this workgroup's rows)
        for (int e = row0 + threadIdx.x; e < min(row0 + RV_ROWS, M); e += 256) Xi[e] = ka.Fc[(size_t)(k - 1) * M + e];
        return;
    }
    const double* Zi = L.Z + i * MM * 2;
    Gemv2 g;
    g.M1 = Zi; g.ld1 = 2 * M;
    g.M2 = Zi + M; g.ld2 = 2 * M;
    g.v1 = k > 0 ? ka.Fc + (size_t)(k - 1) * M : nullptr;
    g.v2 = k < P - 1 ? ka.Fc + (size_t)k * M : nullptr;
    g.base = Xi; g.out = Xi;
    gemv2_rows(g, M, row0 + (threadIdx.x >> 6) * 4, threadIdx.x & 63);
}

// Coupling right-hand side: blockIdx.x separator j (row q = sep[j+1]),
// blockIdx.y its 16-row slice.
__global__ __launch_bounds__(256) void k_couple_rhs_v(const KArgs ka) {
    const Level& L = ka.L;
    const int jj = blockIdx.x, M = L.M, q = L.sep[jj + 1];
    const size_t MM = (size_t)M * M;
    Gemv2 g;
    g.M1 = L.B + q * MM; g.ld1 = M;
    g.M2 = L.C + q * MM; g.ld2 = M;
    g.v1 = ka.X + (size_t)(q - 1) * M;
    g.v2 = ka.X + (size_t)(q + 1) * M;
    g.base = ka.F + (size_t)q * M;
    g.out = ka.Fc + (size_t)jj * M;
    gemv2_rows(g, M, blockIdx.y * RV_ROWS + (threadIdx.x >> 6) * 4, threadIdx.x & 63);
}

// ------------------------------------------------------------------ residual
//
// r = F - (B X_{i-1} + A X_i + C X_{i+1}); per column sum of squares of r
// and of F.  One workgroup per (block row, column); each wave takes whole
// rows, its lanes covering the row in 32-byte pieces (one coalesced read of
// the row of A_i, B_i and C_i per 256 columns), the matching pieces of the
// three X columns held in registers, four rows in flight, and a DPP sum per
// row.  The workgroup writes its partial sums (no atomics: the reduction
// order is fixed); a second kernel sums them.
// rout (optional): the residual vector r itself, [N][M][R].
__global__ __launch_bounds__(256) void k_residual_rows(int N, int M, int R, const double* __restrict__ A,
                                                      const double* __restrict__ B, const double* __restrict__ C,
                                                      const double* __restrict__ X, const double* __restrict__ F,
                                                      double* __restrict__ part, double* __restrict__ rout) {
    const int i = blockIdx.x, c = blockIdx.y;
    const size_t MM = (size_t)M * M, MR = (size_t)M * R;
    __shared__ double sr[4], sf[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool hasb = i > 0, hasc = i < N - 1;
    double accr = 0.0, accf = 0.0;
    if ((M & 255) == 0 && M <= 512) {
        // lane l covers columns 4l..4l+3 of every 256-column piece
        constexpr int MAXP = BTD_MAX_M / 256;
        const int np = M / 256;
        double xa[MAXP][4], xb[MAXP][4], xc[MAXP][4];
#pragma unroll
        for (int q = 0; q < MAXP; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = q * 256 + 4 * lane + e;
                const bool ok = q < np;
                xa[q][e] = ok ? X[i * MR + (size_t)k * R + c] : 0.0;
                xb[q][e] = (ok && hasb) ? X[(i - 1) * MR + (size_t)k * R + c] : 0.0;
                xc[q][e] = (ok && hasc) ? X[(i + 1) * MR + (size_t)k * R + c] : 0.0;
            }
        for (int r0 = w * 4; r0 < M; r0 += 16) {
            double s[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const size_t ro = i * MM + (size_t)(r0 + u) * M + 4 * lane;
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < MAXP; ++q) {
                    if (q < np) {
                        const double4 va = *(const double4*)(A + ro + q * 256);
                        acc = fma(va.x, xa[q][0], acc); acc = fma(va.y, xa[q][1], acc);
                        acc = fma(va.z, xa[q][2], acc); acc = fma(va.w, xa[q][3], acc);
                        if (hasb) {
                            const double4 vb = *(const double4*)(B + ro + q * 256);
                            acc = fma(vb.x, xb[q][0], acc); acc = fma(vb.y, xb[q][1], acc);
                            acc = fma(vb.z, xb[q][2], acc); acc = fma(vb.w, xb[q][3], acc);
                        }
                        if (hasc) {
                            const double4 vc = *(const double4*)(C + ro + q * 256);
                            acc = fma(vc.x, xc[q][0], acc); acc = fma(vc.y, xc[q][1], acc);
                            acc = fma(vc.z, xc[q][2], acc); acc = fma(vc.w, xc[q][3], acc);
                        }
                    }
                }
                s[u] = acc;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double tot = wave_sum(s[u]);
                const double f = F[i * MR + (size_t)(r0 + u) * R + c];
                const double rv = f - tot;
                if (rout && lane == 0) rout[i * MR + (size_t)(r0 + u) * R + c] = rv;
                accr += rv * rv;
                accf += f * f;
            }
        }
    } else {
        for (int row = w; row < M; row += 4) {
            double acc = 0.0;
            for (int kk = lane; kk < M; kk += 64) {
                acc = fma(A[i * MM + (size_t)row * M + kk], X[i * MR + (size_t)kk * R + c], acc);
                if (hasb) acc = fma(B[i * MM + (size_t)row * M + kk], X[(i - 1) * MR + (size_t)kk * R + c], acc);
                if (hasc) acc = fma(C[i * MM + (size_t)row * M + kk], X[(i + 1) * MR + (size_t)kk * R + c], acc);
            }
            const double tot = wave_sum(acc);
            const double f = F[i * MR + (size_t)row * R + c];
            const double rv = f - tot;
            if (rout && lane == 0) rout[i * MR + (size_t)row * R + c] = rv;
            accr += rv * rv;
            accf += f * f;
        }
    }
    if (lane == 0) { sr[w] = accr; sf[w] = accf; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[((size_t)c * N + i) * 2 + 0] = (sr[0] + sr[1]) + (sr[2] + sr[3]);
        part[((size_t)c * N + i) * 2 + 1] = (sf[0] + sf[1]) + (sf[2] + sf[3]);
    }
}

// The same for two or more right-hand sides: one workgroup per (block row, 64-row
// tile of M, 64-column tile of R) forms the 64 x 64 tile of
// A_i X_i + B_i X_{i-1} + C_i X_{i+1} on MFMA (the GEMM tile of the
// factor products, three K sweeps), and writes the tile's per-column sums
// of squares of r and F, reduced in a fixed order through LDS.
constexpr int RES_TILE_MIN_R = 2;   // one column: the row kernel (HBM-bound)

__global__ __launch_bounds__(256) void k_residual_tiles(int N, int M, int R, const double* __restrict__ A,
                                                       const double* __restrict__ B, const double* __restrict__ C,
                                                       const double* __restrict__ X, const double* __restrict__ F,
                                                       double* __restrict__ part, double* __restrict__ rout) {
    __shared__ double As[2 * ASZ];
    __shared__ double Bs[2 * BSZ];
    __shared__ double red[2][4][2][64];   // [r / F][wave][column tile][lane]
    const int ntm = (M + TB - 1) / TB, ntn = (R + TB - 1) / TB;
    int bid = blockIdx.x;
    const int tn = bid % ntn;
    bid /= ntn;
    const int tm = bid % ntm, i = bid / ntm;
    const int row0 = tm * TB, col0 = tn * TB;
    const size_t MM = (size_t)M * M, MR = (size_t)M * R;
    v4d acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = (v4d){0.0, 0.0, 0.0, 0.0};
    tile_accumulate(A + i * MM, M, X + i * MR, R, M, row0, col0, M, R, acc, As, Bs);
    if (i > 0) tile_accumulate(B + i * MM, M, X + (i - 1) * MR, R, M, row0, col0, M, R, acc, As, Bs);
    if (i < N - 1) tile_accumulate(C + i * MM, M, X + (i + 1) * MR, R, M, row0, col0, M, R, acc, As, Bs);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int col = col0 + wc + 16 * c + (lane & 15);
        double sr = 0.0, sf = 0.0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = row0 + wr + 16 * a + (lane >> 4) + 4 * v;
                if (row < M && col < R) {
                    const double f = F[i * MR + (size_t)row * R + col];
                    const double rv = f - acc[a][c][v];
                    if (rout) rout[i * MR + (size_t)row * R + col] = rv;
                    sr = fma(rv, rv, sr);
                    sf = fma(f, f, sf);
                }
            }
        red[0][w][c][lane] = sr;
        red[1][w][c][lane] = sf;
    }
    __syncthreads();
    if (threadIdx.x < 2 * TB) {
        const int q = threadIdx.x & (TB - 1), k = threadIdx.x >> 6;   // column of the tile, r or F
        const int wq = q >> 5, c = (q >> 4) & 1, l16 = q & 15;
        double sum = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int g = 0; g < 4; ++g) sum += red[k][wq + 2 * h][c][l16 + 16 * g];
        const int col = col0 + q;
        if (col < R) part[(((size_t)col * N + i) * ntm + tm) * 2 + k] = sum;
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

template <int MODE, int NPARTS, class CT = double>
static hipError_t launch_gemm(const KArgs& ka, int batch, int m, int n, hipStream_t s) {
    const int tm = cdiv(m, TB), tn = cdiv(n, TB);
    dim3 grid(tm * tn * NPARTS * batch);
    hipLaunchKernelGGL((k_gemm<MODE, NPARTS, CT>), grid, dim3(256), 0, s, ka, tm, tn);
    return hipGetLastError();
}

// ka.lowp: the Schur-complement and spike products of the factor in FP32
// (FP32 MFMA, FP32 accumulation) instead of FP64.
hipError_t launch_fwd_gemm(const KArgs& ka, hipStream_t s) {
    return ka.lowp ? launch_gemm<GM_FWD, 2, float>(ka, ka.nc, ka.L.M, ka.L.M, s)
                   : launch_gemm<GM_FWD, 2>(ka, ka.nc, ka.L.M, ka.L.M, s);
}
hipError_t launch_bwd_gemm(const KArgs& ka, hipStream_t s) {
    return ka.lowp ? launch_gemm<GM_BWD, 2, float>(ka, ka.nc, ka.L.M, ka.L.M, s)
                   : launch_gemm<GM_BWD, 2>(ka, ka.nc, ka.L.M, ka.L.M, s);
}
hipError_t launch_couple(const KArgs& ka, hipStream_t s) { return launch_gemm<GM_COUPLE, 3>(ka, ka.L.P - 1, ka.L.M, ka.L.M, s); }
// The one-column forms need M a multiple of 128 and 32-byte aligned rows.
static bool gemv2_ok(int M, int R, const void* a, const void* b) {
    return R == 1 && M % 128 == 0 && (((uintptr_t)a | (uintptr_t)b) & 31) == 0;
}
hipError_t launch_couple_rhs(const KArgs& ka, hipStream_t s) {
    if (gemv2_ok(ka.L.M, ka.R, ka.L.B, ka.L.C)) {
        hipLaunchKernelGGL(k_couple_rhs_v, dim3(ka.L.P - 1, ka.L.M / RV_ROWS), dim3(256), 0, s, ka);
        return hipGetLastError();
    }
    return launch_gemm<GM_COUPLE_RHS, 1>(ka, ka.L.P - 1, ka.L.M, ka.R, s);
}
hipError_t launch_recover(const KArgs& ka, hipStream_t s) {
    if (gemv2_ok(ka.L.M, ka.R, ka.L.Z, ka.L.Z)) {
        hipLaunchKernelGGL(k_recover_v, dim3(ka.L.N, ka.L.M / RV_ROWS), dim3(256), 0, s, ka);
        return hipGetLastError();
    }
    return launch_gemm<GM_RECOVER, 1>(ka, ka.L.N, ka.L.M, ka.R, s);
}

// One thread per row: 256 threads and 32-column panels up to M = 256,
// 512 threads and 16-column panels above (the LDS holds the multiplier rows
// and U12 of one panel).
static bool getrf_small(int M) { return M <= 256; }

size_t getrf_lds_bytes(int M) {
    return getrf_small(M) ? std::max(lw_lds_layout().total, np_lds_layout().total) : lu_lds_layout(M, 512, 16).total;
}

hipError_t launch_getrf(const KArgs& ka, hipStream_t s) {
    const int M = ka.L.M;
    const size_t lds = getrf_lds_bytes(M);
    dim3 grid(ka.nc);
    if (getrf_small(M)) hipLaunchKernelGGL(k_getrf_pw, grid, dim3(LW_NT), lds, s, ka);
    else hipLaunchKernelGGL((k_getrf<512, 16>), grid, dim3(512), lds, s, ka);
    return hipGetLastError();
}

bool lu_prepares(int M) { return M % DB == 0 && M <= 256; }

hipError_t launch_diag_inv(const KArgs& ka, hipStream_t s) {
    if (lu_prepares(ka.L.M)) return hipSuccess;   // the LU kernel prepared every row
    hipLaunchKernelGGL(k_diag_prep, dim3(cdiv(ka.L.M, DB), ka.nc), dim3(256), 0, s, ka);
    return hipGetLastError();
}

static int slab_width(int M) { return M <= 256 ? 32 : 16; }

template <int NBLK, int NT16, int WPB = 4, bool RHS = false, int WPE = 1>
static void launch_getrs_s(const KArgs& ka, hipStream_t s) {
    const int nslab = cdiv(RHS ? ka.R : 2 * ka.L.M, 16 * NT16), wpc = cdiv(nslab, WPB);
    if (!RHS && ka.lowp)
        hipLaunchKernelGGL((k_getrs_s<NBLK, NT16, WPB, false, float, WPE>), dim3(wpc * ka.nc), dim3(64 * WPB), 0, s,
                           ka, nslab, wpc);
    else
        hipLaunchKernelGGL((k_getrs_s<NBLK, NT16, WPB, RHS, double, WPE>), dim3(wpc * ka.nc), dim3(64 * WPB), 0, s,
                           ka, nslab, wpc);
}

// M <= 256: slabs of 32 columns (64 for M <= 64; 16 above M = 128) held in
// one wave's accumulators, four slabs of one chunk per workgroup sharing the
// factor blocks through LDS (above M = 128 with at most 256 VGPRs, two
// workgroups per CU); above: the workgroup slab kernel.
hipError_t launch_getrs(const KArgs& ka, hipStream_t s) {
    const int M = ka.L.M;
    if (M <= 256) {
        const int nblk = cdiv(M, DB);
        if (nblk <= 1) launch_getrs_s<1, 4>(ka, s);
        else if (nblk <= 2) launch_getrs_s<2, 4>(ka, s);
        else if (nblk <= 4) launch_getrs_s<4, 2>(ka, s);
        else launch_getrs_s<8, 1, 4, false, 2>(ka, s);
        return hipGetLastError();
    }
    const int sw = slab_width(M);
    dim3 grid(cdiv(2 * M, sw) * ka.nc);
    hipLaunchKernelGGL((k_getrs<16, 4>), grid, dim3(256), 0, s, ka);
    return hipGetLastError();
}

// Right-hand-side sweep of many columns as batched steps over all chunks
// (M <= 256): the product X_i = F_i - B_i X_{i-1}, the LU solve of X_i in
// 16-column slabs, and after the forward steps X_i -= E_i X_{i+1}.
bool rhs_batched(int M, int R) { return M <= 256 && R >= 16; }
hipError_t launch_rhs_fwd_gemm(const KArgs& ka, hipStream_t s) { return launch_gemm<GM_RHS_FWD, 1>(ka, ka.nc, ka.L.M, ka.R, s); }
hipError_t launch_rhs_bwd_gemm(const KArgs& ka, hipStream_t s) { return launch_gemm<GM_RHS_BWD, 1>(ka, ka.nc, ka.L.M, ka.R, s); }
hipError_t launch_rhs_getrs(const KArgs& ka, hipStream_t s) {
    const int nblk = cdiv(ka.L.M, DB);
    if (nblk <= 1) launch_getrs_s<1, 1, 4, true>(ka, s);
    else if (nblk <= 2) launch_getrs_s<2, 1, 4, true>(ka, s);
    else if (nblk <= 4) launch_getrs_s<4, 1, 4, true>(ka, s);
    else launch_getrs_s<8, 1, 4, true>(ka, s);
    return hipGetLastError();
}

// Columns per workgroup and staging-panel width of the right-hand-side sweep
// (LDS: three M x RB blocks plus an M x (KC+1) panel).
static int chunk_solve_rb(int M, int R) {
    const int rb = R <= 1 ? 1 : R <= 2 ? 2 : R <= 4 ? 4 : 8;
    return M > 256 && rb > 4 ? 4 : rb;
}
static int chunk_solve_kc(int M) { return M <= 256 ? 32 : 16; }

size_t chunk_solve_lds_bytes(int M, int R) {
    const int rb = chunk_solve_rb(M, R), kc = chunk_solve_kc(M);
    return sizeof(double) * (3 * (size_t)M * rb + (size_t)DB * rb + (size_t)DB * DB + (size_t)M * (kc + 1));
}

template <int KC>
static void launch_chunk_solve_kc(const KArgs& ka, int rb, dim3 grid, size_t lds, hipStream_t s) {
    switch (rb) {
        case 1: hipLaunchKernelGGL((k_chunk_solve<1, KC>), grid, dim3(256), lds, s, ka); break;
        case 2: hipLaunchKernelGGL((k_chunk_solve<2, KC>), grid, dim3(256), lds, s, ka); break;
        case 4: hipLaunchKernelGGL((k_chunk_solve<4, KC>), grid, dim3(256), lds, s, ka); break;
        default: hipLaunchKernelGGL((k_chunk_solve<8, KC>), grid, dim3(256), lds, s, ka); break;
    }
}

// The one-column sweep kernel: R = 1, M a multiple of 64, rows of B 32-byte aligned.
static bool rhs_lean(int M, int R, const void* B) { return R == 1 && M % 64 == 0 && ((uintptr_t)B & 31) == 0; }

static void launch_rhs_sweep1(const KArgs& ka, hipStream_t s) {
    const dim3 grid(ka.L.P), block(256);
    switch (ka.L.M / 64) {
        case 1: hipLaunchKernelGGL(k_rhs_sweep1<1>, grid, block, 0, s, ka); break;
        case 2: hipLaunchKernelGGL(k_rhs_sweep1<2>, grid, block, 0, s, ka); break;
        case 3: hipLaunchKernelGGL(k_rhs_sweep1<3>, grid, block, 0, s, ka); break;
        case 4: hipLaunchKernelGGL(k_rhs_sweep1<4>, grid, block, 0, s, ka); break;
        case 5: hipLaunchKernelGGL(k_rhs_sweep1<5>, grid, block, 0, s, ka); break;
        case 6: hipLaunchKernelGGL(k_rhs_sweep1<6>, grid, block, 0, s, ka); break;
        case 7: hipLaunchKernelGGL(k_rhs_sweep1<7>, grid, block, 0, s, ka); break;
        default: hipLaunchKernelGGL(k_rhs_sweep1<8>, grid, block, 0, s, ka); break;
    }
}

hipError_t launch_chunk_solve(const KArgs& ka, hipStream_t s) {
    const int M = ka.L.M, rb = chunk_solve_rb(M, ka.R);
    if (rhs_lean(ka.L.M, ka.R, ka.L.B)) {
        launch_rhs_sweep1(ka, s);
        return hipGetLastError();
    }
    dim3 grid(ka.L.P, cdiv(ka.R, rb));
    const size_t lds = chunk_solve_lds_bytes(M, ka.R);
    if (chunk_solve_kc(M) == 32) launch_chunk_solve_kc<32>(ka, rb, grid, lds, s);
    else launch_chunk_solve_kc<16>(ka, rb, grid, lds, s);
    return hipGetLastError();
}

hipError_t launch_init_status(unsigned long long* st, hipStream_t s) {
    hipLaunchKernelGGL(k_init_status, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double* F, int N, int M, int R, unsigned long long* st, hipStream_t s) {
    const size_t n = (size_t)N * M * R;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_check_finite, dim3(blocks), dim3(256), 0, s, F, n, M, R, st);
    return hipGetLastError();
}

hipError_t launch_add(double* X, const double* D, size_t n, hipStream_t s) {
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_add, dim3(blocks), dim3(256), 0, s, X, D, n);
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

size_t residual_parts(int N, int M, int R) {
    return (size_t)N * (R >= RES_TILE_MIN_R ? (size_t)cdiv(M, TB) : 1);
}

hipError_t launch_residual(int N, int M, int R, const double* A, const double* B, const double* C, const double* X,
                           const double* F, double* out, double* work, hipStream_t s, double* rout) {
    if (R >= RES_TILE_MIN_R) {
        const int ntm = cdiv(M, TB), ntn = cdiv(R, TB);
        hipLaunchKernelGGL(k_residual_tiles, dim3(N * ntm * ntn), dim3(256), 0, s, N, M, R, A, B, C, X, F, work, rout);
    } else {
        hipLaunchKernelGGL(k_residual_rows, dim3(N, R), dim3(256), 0, s, N, M, R, A, B, C, X, F, work, rout);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_residual_final, dim3(R), dim3(256), 0, s, (int)residual_parts(N, M, R), R, work, out);
    return hipGetLastError();
}

}  // namespace btd

namespace btd {

#ifdef BTD_PHASE_TIMING
hipError_t read_phase_times(unsigned long long* out) {
    hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase), sizeof(unsigned long long) * 16);
    unsigned long long z[16] = {0};
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(g_phase), z, sizeof(z));
    return e;
}
#endif

// Kernels with more than 64 KiB of dynamic LDS must opt in (gfx950 has
// 160 KiB per CU).
hipError_t configure_kernels() {
    const int lds_max = 160 * 1024;
    hipError_t err;
    const void* getrf_kernels[] = {(const void*)k_getrf_pw, (const void*)k_getrf<512, 16>};
    for (const void* f : getrf_kernels) {
        err = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
        if (err != hipSuccess) return err;
    }

    const void* solve_kernels[] = {(const void*)k_chunk_solve<1, 32>, (const void*)k_chunk_solve<2, 32>,
                                   (const void*)k_chunk_solve<4, 32>, (const void*)k_chunk_solve<8, 32>,
                                   (const void*)k_chunk_solve<1, 16>, (const void*)k_chunk_solve<2, 16>,
                                   (const void*)k_chunk_solve<4, 16>, (const void*)k_chunk_solve<8, 16>};
    for (const void* f : solve_kernels) {
        err = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace btd
