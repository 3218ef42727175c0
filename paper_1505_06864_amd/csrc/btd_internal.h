// btd_internal.h -- device-side data layout shared by the host planner and
// the gfx950 kernels of the decomposition-method solver.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/btd.h"

namespace btd {

#define BTD_ERR_SINGULAR_ BTD_ERR_SINGULAR
#define BTD_ERR_NONFINITE_ BTD_ERR_NONFINITE

// One level of the method: a block-tridiagonal system of N rows split into
// P chunks.  Level 0 is the caller's system; level l+1 is the coupling system
// of level l (N' = P-1, A' = Hd, B' = Hb, C' = Hc).  All pointers are device
// pointers; row-major, block i of an [N][M][M] array at i*M*M.
struct Level {
    const double *A, *B, *C;  // [N][M][M]
    double* LU;               // [N][M][M]   LU factors of D_i (unit L below, U on/above the diagonal)
    double* Dw;               // [P][M][M]   per-chunk working copy of the D_i being factored
    double* DI;               // [N][ceil(M/32)][2][32][32] inverses of the 32x32 diagonal blocks of L and U
    double* W;                // [N][M][2M]  [E_i | Y_i]: E_i = D_i^{-1} C_i, Y = forward sweep of the left spike
    double* Z;                // [N][M][2M]  [Z_L | Z_R] spikes (P > 1)
    double *Hd, *Hb, *Hc;     // [P-1][M][M] coupling system (P > 1)
    int* perm;                // [N][M]      row r of P_i D_i is row perm[r] of D_i
    const int* sep;           // [P+1]       sep[0] = -1, sep[k] = separator between chunks k-1 and k, sep[P] = N
    int N, M, P, level;
};

struct KArgs {
    Level L;
    int step;                  // forward step t or backward step s
    int R;                     // RHS columns (solve kernels)
    const double* F;           // [N][M][R] level right-hand side
    double* X;                 // [N][M][R] level solution (may equal F)
    double* Fc;                // [P-1][M][R] coupling right-hand side / solution h
    unsigned long long* status;
    int c0, nc;                // chunks c0 .. c0+nc-1 handled by a chunk-batched launch
    int lowp;                  // 1: products of the level-0 factor sweeps in FP32 (BTD_PREC_F32_REFINE)
};

struct IntChunk {
    static constexpr int CAP = 256;
    int v[CAP];
};

enum GemmMode { GM_FWD = 0, GM_BWD, GM_COUPLE, GM_COUPLE_RHS, GM_RECOVER, GM_RHS_FWD, GM_RHS_BWD };

// For M <= 256 the first step of a chunk runs no forward product (its LU
// reads A_i and its slab solve reads B_i, the seed of the left spike,
// directly) and the backward sweep no first step (the slab solve of a
// chunk's last row writes that row's spikes Z_e = [Y_e | E_e] itself).
inline bool first_step_reads_inputs(int M) { return M <= 256; }
hipError_t launch_fwd_gemm(const KArgs& ka, hipStream_t s);
hipError_t launch_bwd_gemm(const KArgs& ka, hipStream_t s);
hipError_t launch_couple(const KArgs& ka, hipStream_t s);
hipError_t launch_couple_rhs(const KArgs& ka, hipStream_t s);
hipError_t launch_recover(const KArgs& ka, hipStream_t s);
hipError_t launch_getrf(const KArgs& ka, hipStream_t s);
// The LU kernel prepares its rows for the blocked triangular solves itself
// (inverses of the diagonal blocks into DI, off-diagonal blocks scaled) when
// M is a multiple of 32 and at most 256; otherwise launch_diag_inv does.
bool lu_prepares(int M);
hipError_t launch_diag_inv(const KArgs& ka, hipStream_t s);
hipError_t launch_getrs(const KArgs& ka, hipStream_t s);
hipError_t launch_chunk_solve(const KArgs& ka, hipStream_t s);
bool rhs_batched(int M, int R);
hipError_t launch_rhs_fwd_gemm(const KArgs& ka, hipStream_t s);
hipError_t launch_rhs_getrs(const KArgs& ka, hipStream_t s);
hipError_t launch_rhs_bwd_gemm(const KArgs& ka, hipStream_t s);
hipError_t launch_init_status(unsigned long long* st, hipStream_t s);
// Records in *st the smallest (block row, column) of F [N][M][R] that holds a
// NaN or an infinity (code BTD_ERR_NONFINITE); *st is left unchanged otherwise.
hipError_t launch_check_finite(const double* F, int N, int M, int R, unsigned long long* st, hipStream_t s);
hipError_t launch_write_ints(int* dst, const int* host_vals, int count, hipStream_t s);
// Partial sums per column of the residual kernels (their work array holds
// 2 * residual_parts * R doubles).
size_t residual_parts(int N, int M, int R);
// rout (optional, [N][M][R]): also write the residual vector F - A X.
hipError_t launch_residual(int N, int M, int R, const double* A, const double* B, const double* C,
                           const double* X, const double* F, double* out, double* work, hipStream_t s,
                           double* rout = nullptr);
// X += D over n doubles.
hipError_t launch_add(double* X, const double* D, size_t n, hipStream_t s);
size_t getrf_lds_bytes(int M);
hipError_t configure_kernels();

}  // namespace btd
