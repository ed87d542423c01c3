// Workgroup-level dense FP64 linear algebra on global memory (256 threads).
//
// Used by the setup kernels, where one workgroup owns one subdomain (or one column
// chunk of one subdomain) and walks its blocks in order: Cholesky factorisation,
// triangular solves with many right-hand sides, and GEMM updates. Every routine must be
// called by all threads of the workgroup; `lds` must hold kLdsDoubles doubles.
#pragma once

#include "common.hpp"

namespace feti {

constexpr int kLdsDoubles = 2 * 64 * 32;   // 32 KiB

// C[i][j] -= sum_k A[i][k] * B[k][j] for i < m, j < n, k < kk (general strides).
// lower_only: 64x64 output tiles entirely above the diagonal (j > i for all entries)
// are skipped; entries above the diagonal inside diagonal tiles are still updated.
__device__ inline void wg_gemm_sub(int m, int n, int kk, const double* __restrict__ A, long long sai,
                                   long long sak, const double* __restrict__ B, long long sbk,
                                   long long sbn, double* C, long long sci, long long scj,
                                   bool lower_only, double* lds) {
    const int tid = threadIdx.x;
    // FP64 matrix cores: wavefront w takes the 32 x 32 quadrant (rows 32 (w & 1), columns
    // 32 (w >> 1)) of each 64 x 64 tile; lane (mm, g) supplies A[row mm][4s + g] and
    // B[4s + g][column mm] at sub-step s, and holds rows g + 4v, column mm of each 16 x 16 block.
    const int wave = tid >> 6, lane = tid & 63, mm = lane & 15, g = lane >> 4;
    const int wr = 32 * (wave & 1), wc = 32 * (wave >> 1);
    double* As = lds;            // [32][64]
    double* Bs = lds + 32 * 64;  // [32][64]
    for (int i0 = 0; i0 < m; i0 += 64) {
        for (int j0 = 0; j0 < n; j0 += 64) {
            if (lower_only && j0 >= i0 + 64) continue;
            v4d_t acc[2][2];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = v4d_t{0.0, 0.0, 0.0, 0.0};
            for (int k0 = 0; k0 < kk; k0 += 32) {
                for (int e = tid; e < 64 * 32; e += kWG) {
                    int i, k;
                    if (sak == 1) { k = e & 31; i = e >> 5; } else { i = e & 63; k = e >> 6; }
                    As[k * 64 + i] = (i0 + i < m && k0 + k < kk) ? A[(i0 + i) * sai + (k0 + k) * sak] : 0.0;
                    int j, k2;
                    if (sbn == 1) { j = e & 63; k2 = e >> 6; } else { k2 = e & 31; j = e >> 5; }
                    Bs[k2 * 64 + j] = (j0 + j < n && k0 + k2 < kk) ? B[(k0 + k2) * sbk + (j0 + j) * sbn] : 0.0;
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 32; k += 4) {
                    const double* Ar = As + (k + g) * 64;
                    const double* Br = Bs + (k + g) * 64;
                    const double a0 = Ar[wr + mm], a1 = Ar[wr + 16 + mm];
                    const double b0 = Br[wc + mm], b1 = Br[wc + 16 + mm];
                    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
                    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
                }
                __syncthreads();
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = i0 + wr + 16 * x + g + 4 * v, j = j0 + wc + 16 * y + mm;
                        if (i < m && j < n) C[i * sci + j * scj] -= acc[x][y][v];
                    }
        }
    }
    __syncthreads();
}

// In-place lower Cholesky A = L L^T of the leading n x n block (row-major, lda), blocked
// right-looking with 32-column panels. Returns 0, or 1 + the column of the first
// non-positive (or NaN) pivot. Entries above the diagonal are left unspecified.
__device__ inline int wg_potrf(int n, double* A, long long lda, double* lds) {
    const int tid = threadIdx.x;
    for (int k0 = 0; k0 < n; k0 += 32) {
        const int kb = min(32, n - k0);
        for (int jj = 0; jj < kb; ++jj) {
            const int j = k0 + jj;
            __syncthreads();
            const double d = A[j * lda + j];
            if (!(d > 0.0)) return j + 1;  // uniform: every thread read the same value
            const double inv = 1.0 / sqrt(d);
            for (int i = j + 1 + tid; i < n; i += kWG) A[i * lda + j] *= inv;
            __syncthreads();
            if (tid == 0) A[j * lda + j] = sqrt(d);
            const int ncol = k0 + kb - 1 - j;   // panel columns right of j
            if (ncol > 0) {
                const int nrow = n - (j + 1);
                for (int idx = tid; idx < nrow * ncol; idx += kWG) {
                    int i = j + 1 + idx / ncol, l = j + 1 + idx % ncol;
                    if (i >= l) A[i * lda + l] -= A[i * lda + j] * A[l * lda + j];
                }
            }
        }
        __syncthreads();
        const int m = n - k0 - kb;
        if (m > 0) {
            const double* P = A + (long long)(k0 + kb) * lda + k0;
            wg_gemm_sub(m, m, kb, P, lda, 1, P, 1, lda, A + (long long)(k0 + kb) * lda + (k0 + kb), lda, 1,
                        true, lds);
        }
    }
    __syncthreads();
    return 0;
}

// B <- L^{-1} B for lower-triangular L (n x n, row-major ldl, non-zero diagonal) and B with
// ncols columns; element (i, c) of B lives at B[i*sbi + c*sbc]. Left-looking in blocks of RB
// rows (each block's update from the rows above re-reads them, so larger blocks read less); each
// block is finished by one thread per column (no barriers inside the block). lds must hold
// kLdsDoubles doubles for RB = 32 and kLdsTrsm64 for RB = 64.
constexpr int kLdsTrsm64 = 64 * 65 + 64 * 64;
template <int RB = 32>
__device__ inline void wg_trsm_lower(int n, int ncols, const double* __restrict__ L, long long ldl,
                                     double* B, long long sbi, long long sbc, double* lds) {
    static_assert(RB == 32 || RB == 64, "row block");
    const int tid = threadIdx.x;
    for (int c0 = 0; c0 < ncols; c0 += 64) {
        const int nc = min(64, ncols - c0);
        double* Bc = B + c0 * sbc;
        for (int I0 = 0; I0 < n; I0 += RB) {
            const int rb = min(RB, n - I0);
            if (I0 > 0)
                wg_gemm_sub(rb, nc, I0, L + (long long)I0 * ldl, ldl, 1, Bc, sbi, sbc, Bc + I0 * sbi, sbi, sbc,
                            false, lds);
            double* Ld = lds;                   // [RB][RB + 1]
            double* Bd = lds + RB * (RB + 1);   // [RB][64]
            for (int e = tid; e < RB * RB; e += kWG) {
                const int r = e / RB, q = e % RB;
                Ld[r * (RB + 1) + q] = (r < rb && q <= r) ? L[(I0 + r) * ldl + I0 + q] : 0.0;
            }
            for (int e = tid; e < RB * 64; e += kWG) {
                int r, c;
                if (sbc == 1) { c = e & 63; r = e >> 6; } else { r = e % RB; c = e / RB; }
                Bd[r * 64 + c] = (r < rb && c < nc) ? Bc[(I0 + r) * sbi + c * sbc] : 0.0;
            }
            __syncthreads();
            if (tid < nc) {
                for (int r = 0; r < rb; ++r) {
                    double v = Bd[r * 64 + tid];
                    for (int q = 0; q < r; ++q) v -= Ld[r * (RB + 1) + q] * Bd[q * 64 + tid];
                    Bd[r * 64 + tid] = v / Ld[r * (RB + 1) + r];
                }
            }
            __syncthreads();
            for (int e = tid; e < RB * 64; e += kWG) {
                int r, c;
                if (sbc == 1) { c = e & 63; r = e >> 6; } else { r = e % RB; c = e / RB; }
                if (r < rb && c < nc) Bc[(I0 + r) * sbi + c * sbc] = Bd[r * 64 + c];
            }
            __syncthreads();
        }
    }
}

}  // namespace feti
