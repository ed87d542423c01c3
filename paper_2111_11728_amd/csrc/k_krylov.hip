// Block Krylov kernels of the FETI iterations (FP64): Gram products over blocks of
// search directions with two-stage deterministic reductions, the rank-revealing pivoted
// Cholesky of the k x k Gram matrix (Sec. 3.3, Algorithm 1), the F-orthonormalisation of
// the kept directions and the block Gram-Schmidt update against stored directions.
#include "kernels.hpp"

#include <stdexcept>

namespace feti {

constexpr int kGramRows = 32;   // rows staged per LDS step

int gram_chunks(int n, int nblk) {
    return std::max(1, std::min({256, 4096 / std::max(1, nblk), (n + 255) / 256}));
}

// part[(b*nchunk + c)][ka x kb] = A_b[rows of chunk c]^T B[rows of chunk c], ka, kb <= 64.
__global__ void __launch_bounds__(256) k_gram(int n, int ka, int kb, const double* const* __restrict__ Aptrs,
                                              const double* __restrict__ B, double* __restrict__ part) {
    __shared__ double As[kGramRows][64];
    __shared__ double Bs[kGramRows][64];
    const int nchunk = gridDim.x, c = blockIdx.x, b = blockIdx.y;
    const double* A = Aptrs[b];
    const int rows_per = (n + nchunk - 1) / nchunk;
    const int r0 = c * rows_per, r1 = min(n, r0 + rows_per);
    const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int rr = r0; rr < r1; rr += kGramRows) {
        for (int e = tid; e < kGramRows * 64; e += 256) {
            const int q = e >> 6, col = e & 63;
            const int row = rr + q;
            As[q][col] = (row < r1 && col < ka) ? A[(long long)row * ka + col] : 0.0;
            Bs[q][col] = (row < r1 && col < kb) ? B[(long long)row * kb + col] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < kGramRows; ++q) {
            double a[4], bb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[q][tr * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bb[j] = Bs[q][tc * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], bb[j], acc[i][j]);
        }
        __syncthreads();
    }
    double* out = part + (long long)(b * nchunk + c) * ka * kb;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = tr * 4 + i, nn = tc * 4 + j;
            if (m < ka && nn < kb) out[m * kb + nn] = acc[i][j];
        }
}

__global__ void k_gram_reduce(int nchunk, int nblk, int ka, int kb, const double* __restrict__ part,
                              double* __restrict__ out) {
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long per = (long long)ka * kb;
    if (idx >= per * nblk) return;
    const int b = (int)(idx / per);
    const long long e = idx % per;
    double v = 0.0;
    for (int c = 0; c < nchunk; ++c) v += part[(long long)(b * nchunk + c) * per + e];
    out[idx] = v;
}


// ---------------------------------------------------------------------------------------
// Matrix-core (FP64 MFMA 16x16x4) tall-skinny products of the block Gram-Schmidt step.
// Operand layouts of v_mfma_f64_16x16x4f64: A (16x4): lane l holds A[l%16][l/16];
// B (4x16): lane l holds B[l/16][l%16]; D (16x16): lane l holds D[l/16 + 4v][l%16].
typedef double v4d_t __attribute__((ext_vector_type(4)));

// part[(b*nchunk + c)][ka x kb] = A_b[rows of c]^T B[rows of c]. The chunk is walked in
// 64-row tiles staged through LDS; the next tile is loaded into registers while the matrix
// cores work on the current one. Wave w computes rows 16w..16w+15 of the ka x kb result.
__global__ void __launch_bounds__(256) k_gram_mfma(int n, int ka, int kb, const double* const* __restrict__ Aptrs,
                                                   const double* __restrict__ B, double* __restrict__ part) {
    __shared__ double As[64][65];
    __shared__ double Bs[64][65];
    const int nchunk = gridDim.x, c = blockIdx.x, b = blockIdx.y;
    const double* A = Aptrs[b];
    const int rows_per = ((n + nchunk - 1) / nchunk + 63) & ~63;
    const int r0 = c * rows_per, r1 = min(n, r0 + rows_per);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    v4d_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = v4d_t{0.0, 0.0, 0.0, 0.0};
    double ra[16], rb[16];
    auto load = [&](int t0) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, rr = e >> 6, cc = e & 63;
            const int row = t0 + rr;
            ra[u] = (row < r1 && cc < ka) ? A[(long long)row * ka + cc] : 0.0;
            rb[u] = (row < r1 && cc < kb) ? B[(long long)row * kb + cc] : 0.0;
        }
    };
    if (r0 < r1) load(r0);
    for (int t0 = r0; t0 < r1; t0 += 64) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, rr = e >> 6, cc = e & 63;
            As[rr][cc] = ra[u];
            Bs[rr][cc] = rb[u];
        }
        __syncthreads();
        if (t0 + 64 < r1) load(t0 + 64);
        if (16 * wave < ka) {
#pragma unroll 4
            for (int k0 = 0; k0 < 64; k0 += 4) {
                const double a = As[k0 + (lane >> 4)][16 * wave + (lane & 15)];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double bv = Bs[k0 + (lane >> 4)][16 * j + (lane & 15)];
                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[j], 0, 0, 0);
                }
            }
        }
    }
    double* out = part + (long long)(b * nchunk + c) * ka * kb;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * wave + (lane >> 4) + 4 * v, jj = 16 * j + (lane & 15);
            if (i < ka && jj < kb) out[i * kb + jj] = acc[j][v];
        }
}

// out = beta C + alpha sum_b A_b M_b  (A_b: n x kd row-major via Aptrs, M_b = Mats + b*kd*kd,
// C and out n x kd, out may alias C). Workgroup = 64 rows; A_b rows are staged through LDS
// (transposed) so that the A operand is read conflict-free, and the next block is loaded into
// registers while the matrix cores work on the current one; the accumulators stay in
// registers across all blocks b.
__global__ void __launch_bounds__(256) k_ts_gemm(int n, int kd, int nblk, const double* const* __restrict__ Aptrs,
                                                 const double* __restrict__ Mats, const double* C, double* out,
                                                 double alpha, double beta) {
    __shared__ double As[64][65];   // As[col][row]
    __shared__ double Ms[64][64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r0 = blockIdx.x * 64;
    v4d_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = v4d_t{0.0, 0.0, 0.0, 0.0};
    double ra[16], rm[16];
    auto load = [&](int b) {
        const double* A = Aptrs[b];
        const double* Mb = Mats + (long long)b * kd * kd;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, rr = e >> 6, cc = e & 63;
            const int row = r0 + rr;
            ra[u] = (row < n && cc < kd) ? A[(long long)row * kd + cc] : 0.0;
            rm[u] = (rr < kd && cc < kd) ? Mb[rr * kd + cc] : 0.0;
        }
    };
    if (nblk > 0) load(0);
    for (int b = 0; b < nblk; ++b) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + 256 * u, rr = e >> 6, cc = e & 63;
            As[cc][rr] = ra[u];
            Ms[rr][cc] = rm[u];
        }
        __syncthreads();
        if (b + 1 < nblk) load(b + 1);
        for (int k0 = 0; k0 < kd; k0 += 4) {
            const double a = As[k0 + (lane >> 4)][16 * wave + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double bv = Ms[k0 + (lane >> 4)][16 * j + (lane & 15)];
                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[j], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = r0 + 16 * wave + (lane >> 4) + 4 * v, col = 16 * j + (lane & 15);
            if (row < n && col < kd) {
                const long long idx = (long long)row * kd + col;
                out[idx] = (beta == 0.0 ? 0.0 : beta * C[idx]) + alpha * acc[j][v];
            }
        }
}

void launch_ts_gemm(int n, int kd, int nblk, const double* const* Aptrs, const double* Mats, const double* C,
                    double* out, double alpha, double beta, hipStream_t st) {
    if (n && nblk) k_ts_gemm<<<(n + 63) / 64, 256, 0, st>>>(n, kd, nblk, Aptrs, Mats, C, out, alpha, beta);
}

void launch_gram(int n, int ka, int kb, const double* const* Aptrs, int nblk, const double* B, double* part,
                 double* out, hipStream_t st) {
    if (nblk == 0) return;
    const int nchunk = gram_chunks(n, nblk);
    if ((long long)nchunk * nblk * ka * kb > kGramPartCap) throw std::length_error("Gram partial buffer too small");
    if (ka >= 16 && kb >= 16)
        k_gram_mfma<<<dim3(nchunk, nblk), 256, 0, st>>>(n, ka, kb, Aptrs, B, part);
    else
        k_gram<<<dim3(nchunk, nblk), 256, 0, st>>>(n, ka, kb, Aptrs, B, part);
    const long long tot = (long long)ka * kb * nblk;
    k_gram_reduce<<<(int)((tot + 255) / 256), 256, 0, st>>>(nchunk, nblk, ka, kb, part, out);
}

// ---------------------------------------------------------------------------------------
// Rank-revealing Cholesky of the k x k Gram matrix D = Q^T W (one wavefront).
// Jacobi scaling Dhat = S^{-1/2} D S^{-1/2}; columns with D_jj <= 1e-30 max D_jj are
// excluded; outer-product Cholesky with diagonal pivoting (largest remaining Schur-
// complement diagonal, lowest index on ties), stopping when that pivot is <= rr_tol.
// Output T = S^{-1/2} N^T [Ltilde^{-T}; 0] (k x k row-major, zero columns beyond the rank)
// so that W T is F-orthonormal, and the rank.
__global__ void __launch_bounds__(64) k_pivchol(int k, const double* __restrict__ D, double rr_tol,
                                                double* __restrict__ T, int* __restrict__ rank_out) {
    __shared__ double A[64][65];
    __shared__ double L[64][65];   // L[m][l]: column m of the factor, indexed by original index l
    __shared__ double X[64][65];
    __shared__ int order[64];
    __shared__ double scs[64];
    const int l = threadIdx.x;
    for (int i = 0; i < k; ++i)
        if (l < k) A[i][l] = 0.5 * (D[i * k + l] + D[l * k + i]);
    __syncthreads();
    double dg = l < k ? A[l][l] : -1.0;
    double dmax = dg;
    for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
    const bool live = l < k && dmax > 0.0 && dg > 1e-30 * dmax;
    const double sc = live ? 1.0 / sqrt(dg) : 0.0;
    scs[l] = sc;
    __syncthreads();
    // scale: lane l owns column l
    for (int i = 0; i < k; ++i)
        if (l < k) A[i][l] = A[i][l] * scs[i] * sc;
    __syncthreads();
    bool rem = live;
    int m = 0;
    for (; m < k; ++m) {
        double cand = rem ? A[l][l] : -1.0e300;
        int ci = l;
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(cand, o, 64);
            const int oi = __shfl_xor(ci, o, 64);
            if (ov > cand || (ov == cand && oi < ci)) { cand = ov; ci = oi; }
        }
        if (!(cand > rr_tol)) break;
        const int p = ci;
        const double piv = sqrt(cand);
        const double lc = (l == p) ? piv : (rem ? A[l][p] / piv : 0.0);
        if (l == p) rem = false;
        if (l < 64) L[m][l] = lc;
        if (l == 0) order[m] = p;
        __syncthreads();
        // Schur-complement update of the remaining columns: A[i][l] -= lc_i lc_l
        if (rem)
            for (int i = 0; i < k; ++i) A[i][l] -= L[m][i] * lc;
        __syncthreads();
    }
    const int rank = m;
    // Ltilde[r][c] = L[c][order[r]] (rank x rank lower); X = Ltilde^{-1}, lane c owns column c
    if (l < rank) {
        for (int r = 0; r < rank; ++r) {
            double v = (r == l) ? 1.0 : 0.0;
            for (int q = 0; q < r; ++q) v -= L[q][order[r]] * X[q][l];
            X[r][l] = v / L[r][order[r]];
        }
    }
    __syncthreads();
    for (int i = 0; i < k; ++i)
        if (l < k) T[i * k + l] = 0.0;
    __syncthreads();
    // T[order[r]][c] = s[order[r]] * (Ltilde^{-T})[r][c] = s[order[r]] * X[c][r]
    if (l < rank)
        for (int r = 0; r < rank; ++r) T[order[r] * k + l] = scs[order[r]] * X[l][r];
    if (l == 0) *rank_out = rank;
}

void launch_pivchol(int k, const double* D, double rr_tol, double* T, int* rank, hipStream_t st) {
    k_pivchol<<<1, 64, 0, st>>>(k, D, rr_tol, T, rank);
}

// Wo = W T, Qo = Q T (n x k by k x k), 4 rows x 64 columns per workgroup step.
__global__ void __launch_bounds__(256) k_apply_T(int n, int k, const double* __restrict__ Tm,
                                                 const double* __restrict__ W, const double* __restrict__ Q,
                                                 double* __restrict__ Wo, double* __restrict__ Qo) {
    __shared__ double Ts[64][65];
    __shared__ double Ws[4][64], Qs[4][64];
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int i = e >> 6, j = e & 63;
        Ts[i][j] = (i < k && j < k) ? Tm[i * k + j] : 0.0;
    }
    const int rl = threadIdx.x >> 6, c = threadIdx.x & 63;
    for (int r0 = blockIdx.x * 64; r0 < min(n, blockIdx.x * 64 + 64); r0 += 4) {
        __syncthreads();
        const int row = r0 + rl;
        Ws[rl][c] = (row < n && c < k) ? W[(long long)row * k + c] : 0.0;
        Qs[rl][c] = (row < n && c < k) ? Q[(long long)row * k + c] : 0.0;
        __syncthreads();
        if (row < n && c < k) {
            double aw = 0.0, aq = 0.0;
            for (int q = 0; q < k; ++q) {
                aw += Ws[rl][q] * Ts[q][c];
                aq += Qs[rl][q] * Ts[q][c];
            }
            Wo[(long long)row * k + c] = aw;
            Qo[(long long)row * k + c] = aq;
        }
    }
}

void launch_apply_T(int n, int k, const double* T, const double* W, const double* Q, double* Wo, double* Qo,
                    hipStream_t st) {
    if (n) k_apply_T<<<(n + 63) / 64, 256, 0, st>>>(n, k, T, W, Q, Wo, Qo);
}

// lam += W g; r -= Q g (one thread per row).
__global__ void k_update_lr(int n, int k, const double* __restrict__ W, const double* __restrict__ Q,
                            const double* __restrict__ g, double* __restrict__ lam, double* __restrict__ r) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    double dl = 0.0, dr = 0.0;
    for (int q = 0; q < k; ++q) {
        dl += W[(long long)row * k + q] * g[q];
        if (Q) dr += Q[(long long)row * k + q] * g[q];
    }
    lam[row] += dl;
    if (Q) r[row] -= dr;
}

void launch_update_lr(int n, int k, const double* W, const double* Q, const double* g, double* lam, double* r,
                      hipStream_t st) {
    if (n) k_update_lr<<<(n + 255) / 256, 256, 0, st>>>(n, k, W, Q, g, lam, r);
}

// W -= sum_b W_b Psi_b, Psi_b = Psi + b*k*k (k x k), W_b = Wptrs[b] (n x k).
__global__ void __launch_bounds__(256) k_orth_update(int n, int k, const double* const* __restrict__ Wptrs, int nblk,
                                                     const double* __restrict__ Psi, double* __restrict__ W) {
    __shared__ double Ps[64][64];
    __shared__ double Bs[32][64];
    const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const int r0 = blockIdx.x * 32;
    double acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0;
    for (int b = 0; b < nblk; ++b) {
        __syncthreads();
        const double* Wb = Wptrs[b];
        const double* Pb = Psi + (long long)b * k * k;
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int i = e >> 6, j = e & 63;
            Ps[i][j] = (i < k && j < k) ? Pb[i * k + j] : 0.0;
            if (i < 32) {
                const int row = r0 + i;
                Bs[i][j] = (row < n && j < k) ? Wb[(long long)row * k + j] : 0.0;
            }
        }
        __syncthreads();
        for (int q = 0; q < k; ++q) {
            const double p = Ps[q][c];
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] += Bs[rg + 4 * i][q] * p;
        }
    }
    if (c < k)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int row = r0 + rg + 4 * i;
            if (row < n) W[(long long)row * k + c] -= acc[i];
        }
}

void launch_orth_update(int n, int k, const double* const* Wptrs, int nblk, const double* Psi, double* W,
                        hipStream_t st) {
    if (n && nblk) k_orth_update<<<(n + 31) / 32, 256, 0, st>>>(n, k, Wptrs, nblk, Psi, W);
}

// out = sum_row r[row] * sum_c Z[row][c]  (two-stage, deterministic)
__global__ void __launch_bounds__(256) k_rowsum_dot(int n, int k, const double* __restrict__ r,
                                                    const double* __restrict__ Z, double* __restrict__ part) {
    __shared__ double red[4];
    double v = 0.0;
    for (int row = blockIdx.x * 256 + threadIdx.x; row < n; row += gridDim.x * 256) {
        double z = 0.0;
        for (int c = 0; c < k; ++c) z += Z[(long long)row * k + c];
        v += r[row] * z;
    }
    v = warp_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_sum(int n, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double v = 0.0;
        for (int i = 0; i < n; ++i) v += part[i];
        *out = v;
    }
}

void launch_rowsum_dot(int n, int k, const double* r, const double* Z, double* part, double* out, hipStream_t st) {
    const int nb = std::max(1, std::min(256, (n + 255) / 256));
    k_rowsum_dot<<<nb, 256, 0, st>>>(n, k, r, Z, part);
    k_sum<<<1, 64, 0, st>>>(nb, part, out);
}

__global__ void k_axpby(long long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

void launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t st) {
    if (n) k_axpby<<<(int)((n + 255) / 256), 256, 0, st>>>(n, a, x, b, y);
}

// PCG step with device scalars sc = {a}: lam += a w; r -= a q.
__global__ void k_pcg_update(int n, const double* __restrict__ sc, const double* __restrict__ w,
                             const double* __restrict__ q, double* __restrict__ lam, double* __restrict__ r) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = sc[0];
    lam[i] += a * w[i];
    r[i] -= a * q[i];
}

void launch_pcg_update(int n, const double* sc, const double* w, const double* q, double* lam, double* r,
                       hipStream_t st) {
    if (n) k_pcg_update<<<(n + 255) / 256, 256, 0, st>>>(n, sc, w, q, lam, r);
}

// w = z + beta w with sc = {., beta}
__global__ void k_pcg_dir(int n, const double* __restrict__ sc, const double* __restrict__ z, double* __restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = z[i] + sc[1] * w[i];
}

void launch_pcg_dir(int n, const double* sc, const double* z, double* w, hipStream_t st) {
    if (n) k_pcg_dir<<<(n + 255) / 256, 256, 0, st>>>(n, sc, z, w);
}

}  // namespace feti
