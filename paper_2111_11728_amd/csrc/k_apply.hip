// Application of the dual operator F to a block of search directions (Sec. 2.1 Eq. 7,
// Sec. 2.2 Eq. 12 with u_c condensed), the preconditioner of Sec. 3.1 Eq. (13) and the
// TFETI projector.
//
// F * Lambda = sum_s B^s F_s B^sT Lambda runs in three launches:
//   1. k_flambda: per (subdomain, 128-row tile) gather X_s = B^sT Lambda into LDS (in MFMA
//      operand order) and multiply by the augmented operator A_s = [F_s; F_rc^sT] on the
//      matrix cores; A_s streams from HBM in a pre-swizzled layout so that every wavefront
//      load is one coalesced 16-byte access per lane with no LDS round trip.
//   2. k_coarse (FETI-DP): t = sum_s B_c^sT F_rc^sT X_s, v = Kbar_cc^{-1} t.
//   3. k_scatter: owner-computes per lambda row, Q[row] = sum over the row's (one or two)
//      subdomains of sign * (Y_s[j] + F_rc^s[j,:] v_s); no atomics, bit-reproducible.
#include "kernels.hpp"

namespace feti {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kKC = 64;        // rows of X staged per LDS chunk
constexpr int kTileRows = 128; // rows of A_s per workgroup (4 wavefronts x 32 rows)

template <int P> struct PrecTraits;
template <> struct PrecTraits<FETI_FP64> { typedef double Elem; typedef double Out; };
template <> struct PrecTraits<FETI_FP32> { typedef float Elem; typedef float Out; };
template <> struct PrecTraits<FETI_BF16X3> { typedef __bf16 Elem; typedef float Out; };

__device__ inline __bf16 to_bf16(float x) {
    __hip_bfloat16 h = __float2bfloat16(x);
    return *reinterpret_cast<__bf16*>(&h);
}
__device__ inline float from_bf16(__bf16 x) { return __bfloat162float(*reinterpret_cast<__hip_bfloat16*>(&x)); }

template <int P>
__global__ void __launch_bounds__(256) k_flambda(const SubMeta* __restrict__ subs, const int* __restrict__ tile_sub,
                                                 const int* __restrict__ tile_row, int k,
                                                 const double* __restrict__ Lambda, const int* __restrict__ bg_ptr,
                                                 const int* __restrict__ bg_row, const int8_t* __restrict__ bg_sg,
                                                 const void* __restrict__ Fsw_, const void* __restrict__ Fsw_lo_,
                                                 typename PrecTraits<P>::Out* __restrict__ Y,
                                                 typename PrecTraits<P>::Out* __restrict__ T) {
    typedef typename PrecTraits<P>::Out Out;
    constexpr bool kBF = P == FETI_BF16X3;
    // FP32/FP64: 4 super-blocks of 16 k x 4 column blocks x 64 lanes x 4 values;
    // BF16: 2 blocks of 32 k x 4 column blocks x 64 lanes x 8 values (hi and lo)
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[kBF ? 2 * 4096 * 2 : 4096 * sizeof(typename PrecTraits<P>::Elem)];
    const int s = tile_sub[blockIdx.x];
    if (s < 0) return;
    const SubMeta M = subs[s];
    const int row0 = tile_row[blockIdx.x];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int rbase = row0 + 32 * wave;     // first row of this wavefront
    const int rb0 = rbase >> 4;             // first 16-row block
    const int nrb = M.rows_F >> 4;
    const bool rvalid[2] = {rb0 < nrb, rb0 + 1 < nrb};

    typedef typename std::conditional<P == FETI_FP64, v4d, v4f>::type Acc;
    Acc acc[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[r][nb][v] = 0;

    for (int kc0 = 0; kc0 < M.ldF; kc0 += kKC) {
        const int kcn = min(kKC, M.ldF - kc0);   // multiple of 32
        // ---- gather X rows kc0..kc0+kcn (b DOFs) x 64 columns into operand order ----
        for (int e = tid; e < kKC * 64; e += 256) {
            const int jj = e >> 6, c = e & 63;
            const int j = kc0 + jj;
            double val = 0.0;
            if (jj < kcn && j < M.n_b && c < k) {
                const long long q = M.off_b + j;
                for (int en = bg_ptr[q]; en < bg_ptr[q + 1]; ++en)
                    val += bg_sg[en] * Lambda[(long long)bg_row[en] * k + c];
            }
            if constexpr (!kBF) {
                typedef typename PrecTraits<P>::Elem E;
                E* X = reinterpret_cast<E*>(lds_raw);
                const int kq = jj >> 4, q4 = (jj & 15) >> 2, lr = jj & 3;
                const int l = lr * 16 + (c & 15), nb = c >> 4;
                X[((kq * 4 + nb) * 64 + l) * 4 + q4] = (E)val;
            } else {
                __bf16* Xh = reinterpret_cast<__bf16*>(lds_raw);
                __bf16* Xl = Xh + 4096;
                const int kb = jj >> 5, r32 = jj & 31, lg = r32 >> 3, q8 = r32 & 7;
                const int l = lg * 16 + (c & 15), nb = c >> 4;
                const float vf = (float)val;
                const __bf16 hi = to_bf16(vf);
                const __bf16 lo = to_bf16(vf - from_bf16(hi));
                const int idx = ((kb * 4 + nb) * 64 + l) * 8 + q8;
                Xh[idx] = hi;
                Xl[idx] = lo;
            }
        }
        __syncthreads();
        // ---- matrix-core products ----
        if constexpr (P == FETI_FP64 || P == FETI_FP32) {
            typedef typename PrecTraits<P>::Elem E;
            const E* A = reinterpret_cast<const E*>(Fsw_) + M.off_Fsw;
            const E* X = reinterpret_cast<const E*>(lds_raw);
            const int KQ = M.ldF >> 4;
            for (int kq = 0; kq < (kcn >> 4); ++kq) {
                const int kqg = (kc0 >> 4) + kq;
                E a[2][4];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    if (rvalid[r]) {
                        const E* src = A + ((long long)((rb0 + r) * KQ + kqg) * 64 + lane) * 4;
#pragma unroll
                        for (int q = 0; q < 4; ++q) a[r][q] = src[q];
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) a[r][q] = 0;
                    }
                }
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    const E* bsrc = X + ((kq * 4 + nb) * 64 + lane) * 4;
                    E b[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) b[q] = bsrc[q];
#pragma unroll
                    for (int r = 0; r < 2; ++r)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            if constexpr (P == FETI_FP64)
                                acc[r][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r][q], b[q], acc[r][nb], 0, 0, 0);
                            else
                                acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r][q], b[q], acc[r][nb], 0, 0, 0);
                        }
                }
            }
        } else {
            const v8bf* Ah = reinterpret_cast<const v8bf*>(Fsw_) + (M.off_Fsw >> 3);
            const v8bf* Al = reinterpret_cast<const v8bf*>(Fsw_lo_) + (M.off_Fsw >> 3);
            const v8bf* Xh = reinterpret_cast<const v8bf*>(lds_raw);
            const v8bf* Xl = Xh + 512;
            const int KB = M.ldF >> 5;
            for (int kb = 0; kb < (kcn >> 5); ++kb) {
                const int kbg = (kc0 >> 5) + kb;
                v8bf ah[2], al[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    if (rvalid[r]) {
                        const long long idx = (long long)((rb0 + r) * KB + kbg) * 64 + lane;
                        ah[r] = Ah[idx];
                        al[r] = Al[idx];
                    } else {
#pragma unroll
                        for (int q = 0; q < 8; ++q) { ah[r][q] = to_bf16(0.f); al[r][q] = to_bf16(0.f); }
                    }
                }
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) {
                    const int idx = (kb * 4 + nb) * 64 + lane;
                    const v8bf bh = Xh[idx], bl = Xl[idx];
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bh, acc[r][nb], 0, 0, 0);
                        acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bl, acc[r][nb], 0, 0, 0);
                        acc[r][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[r], bh, acc[r][nb], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
    // ---- store: lane holds rows 4*(lane/16)+v, column lane%16 of every 16x16 block ----
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int col = nb * 16 + (lane & 15);
            if (col >= k) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rbase + 16 * r + 4 * (lane >> 4) + v;
                const Out val = (Out)acc[r][nb][v];
                if (row < M.n_b)
                    Y[(M.off_b + row) * k + col] = val;
                else if (row < M.n_b + M.n_c)
                    T[(M.off_c + row - M.n_b) * k + col] = val;
            }
        }
    }
}

void launch_flambda(const DevTopo& t, int precision, int k, const double* Lambda, const void* Fsw,
                    const void* Fsw_lo, void* Y, void* T, hipStream_t st) {
    if (t.n_m_tiles == 0) return;
    dim3 grid(t.n_m_tiles);
    switch (precision) {
        case FETI_FP64:
            k_flambda<FETI_FP64><<<grid, 256, 0, st>>>(t.subs, t.m_tile_sub, t.m_tile_row, k, Lambda, t.bg_ptr,
                                                       t.bg_row, t.bg_sg, Fsw, nullptr, (double*)Y, (double*)T);
            break;
        case FETI_FP32:
            k_flambda<FETI_FP32><<<grid, 256, 0, st>>>(t.subs, t.m_tile_sub, t.m_tile_row, k, Lambda, t.bg_ptr,
                                                       t.bg_row, t.bg_sg, Fsw, nullptr, (float*)Y, (float*)T);
            break;
        default:
            k_flambda<FETI_BF16X3><<<grid, 256, 0, st>>>(t.subs, t.m_tile_sub, t.m_tile_row, k, Lambda, t.bg_ptr,
                                                         t.bg_row, t.bg_sg, Fsw, Fsw_lo, (float*)Y, (float*)T);
            break;
    }
}

// ---------------------------------------------------------------------------------------
// FETI-DP corner coarse problem: t = add + sum_s B_c^sT T_s, v = scale * Kbar_cc^{-1} t.
// Workgroup = 64 coarse rows x 16 columns; t is rebuilt in LDS chunk by chunk.
template <typename TT>
__global__ void __launch_bounds__(256) k_coarse(int n_cg, int k, const TT* __restrict__ T, const double* __restrict__ add,
                                                const int* __restrict__ cc_ptr, const int* __restrict__ cc_s,
                                                const int* __restrict__ cc_j, const SubMeta* __restrict__ subs,
                                                const double* __restrict__ Kinv, double scale, double* v) {
    __shared__ double tc[64][17];
    const int p0 = blockIdx.x * 64, c0 = blockIdx.y * 16;
    const int tid = threadIdx.x;
    const int pr = tid >> 2, cg4 = (tid & 3) * 4;   // row p0+pr, columns c0+cg4..+3
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q0 = 0; q0 < n_cg; q0 += 64) {
        for (int e = tid; e < 64 * 16; e += 256) {
            const int qq = e >> 4, c = e & 15;
            const int q = q0 + qq, col = c0 + c;
            double val = 0.0;
            if (q < n_cg && col < k) {
                if (add) val = add[(long long)q * k + col];
                for (int en = cc_ptr[q]; en < cc_ptr[q + 1]; ++en)
                    val += (double)T[(subs[cc_s[en]].off_c + cc_j[en]) * k + col];
            }
            tc[qq][c] = val;
        }
        __syncthreads();
        const int p = p0 + pr;
        if (p < n_cg) {
            const int qn = min(64, n_cg - q0);
            for (int qq = 0; qq < qn; ++qq) {
                const double kv = Kinv[(long long)p * n_cg + q0 + qq];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] += kv * tc[qq][cg4 + c];
            }
        }
        __syncthreads();
    }
    const int p = p0 + pr;
    if (p < n_cg)
        for (int c = 0; c < 4; ++c)
            if (c0 + cg4 + c < k) v[(long long)p * k + c0 + cg4 + c] = scale * acc[c];
}

void launch_coarse(const DevTopo& t, int k, int ytype_f32, const void* T, const double* add, const double* Kinv,
                   double scale, double* v, hipStream_t st) {
    if (t.n_cg == 0) return;
    dim3 grid((t.n_cg + 63) / 64, (k + 15) / 16);
    if (ytype_f32)
        k_coarse<float><<<grid, 256, 0, st>>>(t.n_cg, k, (const float*)T, add, t.cc_ptr, t.cc_s, t.cc_j, t.subs, Kinv,
                                              scale, v);
    else
        k_coarse<double><<<grid, 256, 0, st>>>(t.n_cg, k, (const double*)T, add, t.cc_ptr, t.cc_s, t.cc_j, t.subs,
                                               Kinv, scale, v);
}

// Q[row][c] = sum over the row's sides of sign * (Y_s[j][c] + sum_q F_rc^s[j][q] v[cg(s,q)][c]).
template <typename TY>
__global__ void k_scatter(int n_lambda, int k, const int* __restrict__ row_s, const int* __restrict__ row_j,
                          const int8_t* __restrict__ row_sg, const SubMeta* __restrict__ subs,
                          const TY* __restrict__ Y, const double* __restrict__ F64, const int* __restrict__ c_glob,
                          const double* __restrict__ v, double* __restrict__ Q) {
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)n_lambda * k) return;
    const int row = (int)(idx / k), c = (int)(idx % k);
    double val = 0.0;
    for (int t = 0; t < 2; ++t) {
        const int s = row_s[2 * row + t];
        if (s < 0) continue;
        const int j = row_j[2 * row + t];
        const SubMeta& M = subs[s];
        double y = (double)Y[(M.off_b + j) * k + c];
        if (v) {
            const double* Fr = F64 + M.off_F + (long long)M.n_b * M.ldF + j;
            for (int q = 0; q < M.n_c; ++q) y += Fr[(long long)q * M.ldF] * v[(long long)c_glob[M.off_c + q] * k + c];
        }
        val += row_sg[2 * row + t] * y;
    }
    Q[idx] = val;
}

void launch_scatter(const DevTopo& t, int k, int ytype_f32, const void* Y, const double* F64, const double* v,
                    double* Q, hipStream_t st) {
    const long long n = (long long)t.n_lambda * k;
    if (n == 0) return;
    const int grid = (int)((n + 255) / 256);
    if (ytype_f32)
        k_scatter<float><<<grid, 256, 0, st>>>(t.n_lambda, k, t.row_s, t.row_j, t.row_sg, t.subs, (const float*)Y, F64,
                                               t.c_glob, v, Q);
    else
        k_scatter<double><<<grid, 256, 0, st>>>(t.n_lambda, k, t.row_s, t.row_j, t.row_sg, t.subs, (const double*)Y,
                                                F64, t.c_glob, v, Q);
}

// ---------------------------------------------------------------------------------------
// Preconditioner (Sec. 3.1, Eq. 13): x_s = B~^sT r = B^sT W^s r, y_s = S~^s x_s.
// One workgroup per (subdomain, 64 rows of S~^s); x_s is gathered whole into LDS.
template <typename TP>
__global__ void __launch_bounds__(256) k_precond_local(const SubMeta* __restrict__ subs, const int* __restrict__ bg_ptr,
                                                       const int* __restrict__ bg_row, const int8_t* __restrict__ bg_sg,
                                                       const double* __restrict__ bg_w, const double* __restrict__ r,
                                                       const TP* __restrict__ P, double* __restrict__ y) {
    extern __shared__ double xs[];
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int j0 = blockIdx.x * 64;
    if (j0 >= M.n_b) return;
    for (int j = threadIdx.x; j < M.n_b; j += 256) {
        const long long q = M.off_b + j;
        double v = 0.0;
        for (int e = bg_ptr[q]; e < bg_ptr[q + 1]; ++e) v += bg_sg[e] * bg_w[e] * r[bg_row[e]];
        xs[j] = v;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int jr = wave; jr < 64; jr += 4) {
        const int j = j0 + jr;
        if (j >= M.n_b) break;
        const TP* Pr = P + M.off_P + (long long)j * M.n_b;
        double acc = 0.0;
        for (int q = lane; q < M.n_b; q += 64) acc += (double)Pr[q] * xs[q];
        acc = warp_sum(acc);
        if (lane == 0) y[M.off_b + j] = acc;
    }
}

void launch_precond_local(const DevTopo& t, int use_f32, const double* r, const double* bg_w, const double* P64,
                          const float* P32, double* y, hipStream_t st) {
    dim3 grid((t.max_nb + 63) / 64, t.n_sub);
    const size_t sh = sizeof(double) * std::max(1, t.max_nb);
    if (use_f32)
        k_precond_local<float><<<grid, 256, sh, st>>>(t.subs, t.bg_ptr, t.bg_row, t.bg_sg, bg_w, r, P32, y);
    else
        k_precond_local<double><<<grid, 256, sh, st>>>(t.subs, t.bg_ptr, t.bg_row, t.bg_sg, bg_w, r, P64, y);
}

// Z[row][c] = sum over the row's sides with g(s) == c of sign * w * y_s[j]  (kz = n_groups or 1).
__global__ void k_precond_scatter(int n_lambda, int kz, int one_column, const int* __restrict__ row_s,
                                  const int* __restrict__ row_j, const int8_t* __restrict__ row_sg,
                                  const SubMeta* __restrict__ subs, const double* __restrict__ w,
                                  const double* __restrict__ y, double* __restrict__ Z) {
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)n_lambda * kz) return;
    const int row = (int)(idx / kz), c = (int)(idx % kz);
    double val = 0.0;
    for (int t = 0; t < 2; ++t) {
        const int s = row_s[2 * row + t];
        if (s < 0) continue;
        const SubMeta& M = subs[s];
        if (!one_column && M.grp != c) continue;
        val += row_sg[2 * row + t] * w[2 * row + t] * y[M.off_b + row_j[2 * row + t]];
    }
    Z[idx] = val;
}

void launch_precond_scatter(const DevTopo& t, int one_column, const double* w, const double* y, double* Z,
                            hipStream_t st) {
    const int kz = one_column ? 1 : t.n_groups;
    const long long n = (long long)t.n_lambda * kz;
    if (n == 0) return;
    k_precond_scatter<<<(int)((n + 255) / 256), 256, 0, st>>>(t.n_lambda, kz, one_column, t.row_s, t.row_j, t.row_sg,
                                                              t.subs, w, y, Z);
}

// ---------------------------------------------------------------------------------------
// TFETI projector P = I - G^T (G G^T)^{-1} G with G = -Rhat^T B^T (Sec. 3.3).
// GY[(s, m)][c] = -sum_j Rhat_s[j][m] (B^sT Y)[j][c].
__global__ void __launch_bounds__(256) k_proj_G(const SubMeta* __restrict__ subs, int nm, int k,
                                                const int* __restrict__ bg_ptr, const int* __restrict__ bg_row,
                                                const int8_t* __restrict__ bg_sg, const double* __restrict__ Y,
                                                const double* __restrict__ Rb, double* GY) {
    __shared__ double red[4][6][64];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    const int c = threadIdx.x & 63, jg = threadIdx.x >> 6;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (c < k) {
        for (int j = jg; j < M.n_b; j += 4) {
            const long long q = M.off_b + j;
            double x = 0.0;
            for (int e = bg_ptr[q]; e < bg_ptr[q + 1]; ++e) x += bg_sg[e] * Y[(long long)bg_row[e] * k + c];
            for (int m = 0; m < nm; ++m) acc[m] += Rb[M.off_R + (long long)j * nm + m] * x;
        }
    }
    for (int m = 0; m < nm; ++m) red[jg][m][c] = acc[m];
    __syncthreads();
    if (jg == 0 && c < k)
        for (int m = 0; m < nm; ++m)
            GY[(long long)(s * nm + m) * k + c] = -(red[0][m][c] + red[1][m][c] + red[2][m][c] + red[3][m][c]);
}

void launch_proj_G(const DevTopo& t, int k, const double* Y, const double* Rb, double* GY, hipStream_t st) {
    k_proj_G<<<t.n_sub, 256, 0, st>>>(t.subs, t.n_rbm, k, t.bg_ptr, t.bg_row, t.bg_sg, Y, Rb, GY);
}

__global__ void k_small_gemm(int m, int n, int kk, const double* __restrict__ A, const double* __restrict__ B,
                             double* __restrict__ C, double alpha) {
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    double v = 0.0;
    for (int q = 0; q < kk; ++q) v += A[(long long)i * kk + q] * B[(long long)q * n + j];
    C[idx] = alpha * v;
}

void launch_small_gemm(int m, int n, int kk, const double* A, const double* B, double* C, double alpha,
                       hipStream_t st) {
    const long long tot = (long long)m * n;
    if (tot) k_small_gemm<<<(int)((tot + 255) / 256), 256, 0, st>>>(m, n, kk, A, B, C, alpha);
}

// Y[row][c] += sign * sum over sides of sg * sum_m Rhat_s[j][m] tcoef[(s, m)][c]
__global__ void k_proj_apply(int n_lambda, int k, int nm, const int* __restrict__ row_s, const int* __restrict__ row_j,
                             const int8_t* __restrict__ row_sg, const SubMeta* __restrict__ subs,
                             const double* __restrict__ tcoef, const double* __restrict__ Rb, double sign,
                             double* __restrict__ Y) {
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)n_lambda * k) return;
    const int row = (int)(idx / k), c = (int)(idx % k);
    double val = 0.0;
    for (int t = 0; t < 2; ++t) {
        const int s = row_s[2 * row + t];
        if (s < 0) continue;
        const SubMeta& M = subs[s];
        const int j = row_j[2 * row + t];
        double d = 0.0;
        for (int m = 0; m < nm; ++m) d += Rb[M.off_R + (long long)j * nm + m] * tcoef[(long long)(s * nm + m) * k + c];
        val += row_sg[2 * row + t] * d;
    }
    Y[idx] += sign * val;
}

void launch_proj_apply(const DevTopo& t, int k, const double* tcoef, const double* Rb, double sign, double* Y,
                       hipStream_t st) {
    const long long n = (long long)t.n_lambda * k;
    if (n) k_proj_apply<<<(int)((n + 255) / 256), 256, 0, st>>>(t.n_lambda, k, t.n_rbm, t.row_s, t.row_j, t.row_sg,
                                                               t.subs, tcoef, Rb, sign, Y);
}

}  // namespace feti
