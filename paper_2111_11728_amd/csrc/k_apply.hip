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

// Gather of X_s = B^sT Lambda rows through the fixed-width map gmap[q*R + t] = sign*(row+1)
// (0: unused slot). Each thread owns kGatherPer (row, column) pairs of a 64-row chunk:
// e = tid + kFLThreads*u, chunk row e/64, column e%64 (a wavefront shares the row: the map
// load is a broadcast and the Lambda loads are one coalesced 512-byte access).
constexpr int kFLThreads = 512;                  // 8 wavefronts x 16 rows = one 128-row tile
constexpr int kGatherPer = kKC * 64 / kFLThreads;

__device__ inline void gather_chunk(const SubMeta& M, int kc0, int kcn, int k, int R, const int* __restrict__ gmap,
                                    const double* __restrict__ Lambda, double* vals) {
#pragma unroll
    for (int u = 0; u < kGatherPer; ++u) {
        const int e = threadIdx.x + kFLThreads * u;
        const int jj = e >> 6, c = e & 63;
        const int j = kc0 + jj;
        double v = 0.0;
        if (jj < kcn && j < M.n_b && c < k) {
            const int* g = gmap + (M.off_b + j) * R;
            for (int t = 0; t < R; ++t) {
                const int gv = g[t];
                if (gv > 0) v += Lambda[(long long)(gv - 1) * k + c];
                else if (gv < 0) v -= Lambda[(long long)(-gv - 1) * k + c];
            }
        }
        vals[u] = v;
    }
}

template <int P>
__device__ inline void store_chunk(unsigned char* lds_raw, const double* vals) {
#pragma unroll
    for (int u = 0; u < kGatherPer; ++u) {
        const int e = threadIdx.x + kFLThreads * u;
        const int jj = e >> 6, c = e & 63;
        if constexpr (P != FETI_BF16X3) {
            typedef typename PrecTraits<P>::Elem E;
            E* X = reinterpret_cast<E*>(lds_raw);
            const int kq = jj >> 4, q4 = (jj & 15) >> 2, lr = jj & 3;
            const int l = lr * 16 + (c & 15), nb = c >> 4;
            X[((kq * 4 + nb) * 64 + l) * 4 + q4] = (E)vals[u];
        } else {
            __bf16* Xh = reinterpret_cast<__bf16*>(lds_raw);
            __bf16* Xl = Xh + 4096;
            const int kb = jj >> 5, r32 = jj & 31, lg = r32 >> 3, q8 = r32 & 7;
            const int l = lg * 16 + (c & 15), nb = c >> 4;
            const float vf = (float)vals[u];
            const __bf16 hi = to_bf16(vf);
            const __bf16 lo = to_bf16(vf - from_bf16(hi));
            const int idx = ((kb * 4 + nb) * 64 + l) * 8 + q8;
            Xh[idx] = hi;
            Xl[idx] = lo;
        }
    }
}

template <int P, typename Out>
__global__ void __launch_bounds__(kFLThreads) k_flambda(const SubMeta* __restrict__ subs, const int* __restrict__ tile_sub,
                                                        const int* __restrict__ tile_row, const int* __restrict__ tile_end,
                                                        int k, const double* __restrict__ Lambda,
                                                        const int* __restrict__ gmap, int R,
                                                        const void* __restrict__ Fsw_, const void* __restrict__ Fsw_lo_,
                                                        Out* __restrict__ Y, Out* __restrict__ T) {
    constexpr bool kBF = P == FETI_BF16X3;
    // FP32/FP64: 4 super-blocks of 16 k x 4 column blocks x 64 lanes x 4 values;
    // BF16: 2 blocks of 32 k x 4 column blocks x 64 lanes x 8 values (hi and lo)
    __shared__ __attribute__((aligned(16))) unsigned char lds_raw[kBF ? 2 * 4096 * 2 : 4096 * sizeof(typename PrecTraits<P>::Elem)];
    const int s = tile_sub[blockIdx.x];
    if (s < 0) return;
    const SubMeta M = subs[s];
    const int row0 = tile_row[blockIdx.x];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int rbase = row0 + 16 * wave;     // first row of this wavefront (one 16-row block)
    const int rb = rbase >> 4;
    const bool rvalid = rb < (min(M.rows_F, tile_end[blockIdx.x]) >> 4);

    typedef typename std::conditional<P == FETI_FP64, v4d, v4f>::type Acc;
    Acc acc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[nb][v] = 0;

    double vals[kGatherPer];
    gather_chunk(M, 0, min(kKC, M.ldF), k, R, gmap, Lambda, vals);
    for (int kc0 = 0; kc0 < M.ldF; kc0 += kKC) {
        const int kcn = min(kKC, M.ldF - kc0);   // multiple of 32
        store_chunk<P>(lds_raw, vals);
        __syncthreads();
        // prefetch the next chunk's gathered values while the matrix cores work on this one
        if (kc0 + kKC < M.ldF) gather_chunk(M, kc0 + kKC, min(kKC, M.ldF - kc0 - kKC), k, R, gmap, Lambda, vals);
        if (rvalid) {
            if constexpr (P == FETI_FP64 || P == FETI_FP32) {
                typedef typename PrecTraits<P>::Elem E;
                const E* A = reinterpret_cast<const E*>(Fsw_) + M.off_Fsw;
                const E* X = reinterpret_cast<const E*>(lds_raw);
                const int KQ = M.ldF >> 4;
                const int nkq = kcn >> 4;
                E a[4][4];
#pragma unroll
                for (int kq = 0; kq < 4; ++kq) {
                    const E* src = A + ((long long)(rb * KQ + (kc0 >> 4) + kq) * 64 + lane) * 4;
#pragma unroll
                    for (int q = 0; q < 4; ++q) a[kq][q] = kq < nkq ? src[q] : (E)0;
                }
#pragma unroll
                for (int kq = 0; kq < 4; ++kq) {
                    if (kq >= nkq) break;
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) {
                        const E* bsrc = X + ((kq * 4 + nb) * 64 + lane) * 4;
                        E bq[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) bq[q] = bsrc[q];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            if constexpr (P == FETI_FP64)
                                acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kq][q], bq[q], acc[nb], 0, 0, 0);
                            else
                                acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kq][q], bq[q], acc[nb], 0, 0, 0);
                        }
                    }
                }
            } else {
                const v8bf* Ah = reinterpret_cast<const v8bf*>(Fsw_) + (M.off_Fsw >> 3);
                const v8bf* Al = reinterpret_cast<const v8bf*>(Fsw_lo_) + (M.off_Fsw >> 3);
                const v8bf* Xh = reinterpret_cast<const v8bf*>(lds_raw);
                const v8bf* Xl = Xh + 512;
                const int KB = M.ldF >> 5;
                const int nkb = kcn >> 5;
                v8bf ah[2], al[2];
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    if (kb < nkb) {
                        const long long idx = (long long)(rb * KB + (kc0 >> 5) + kb) * 64 + lane;
                        ah[kb] = Ah[idx];
                        al[kb] = Al[idx];
                    } else {
#pragma unroll
                        for (int q = 0; q < 8; ++q) { ah[kb][q] = to_bf16(0.f); al[kb][q] = to_bf16(0.f); }
                    }
                }
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    if (kb >= nkb) break;
#pragma unroll
                    for (int nb = 0; nb < 4; ++nb) {
                        const int idx = (kb * 4 + nb) * 64 + lane;
                        const v8bf bh = Xh[idx], bl = Xl[idx];
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[kb], bh, acc[nb], 0, 0, 0);
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[kb], bl, acc[nb], 0, 0, 0);
                        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[kb], bh, acc[nb], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!rvalid) return;
    // ---- store: in every 16x16 block the lane holds column lane%16 and rows
    // 4*(lane/16)+v (FP32 accumulators) or lane/16+4*v (FP64 accumulators) ----
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        const int col = nb * 16 + (lane & 15);
        if (col >= k) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rin = P == FETI_FP64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
            const int row = rbase + rin;
            const Out val = (Out)acc[nb][v];
            if (row < M.n_b)
                Y[(M.off_b + row) * k + col] = val;
            else if (row >= M.rowT && row < M.rowT + M.n_c)
                T[(M.off_c + row - M.rowT) * k + col] = val;
        }
    }
}

void launch_flambda(const DevTopo& t, int precision, int k, const double* Lambda, const void* Fsw,
                    const void* Fsw_lo, void* Y, void* T, hipStream_t st, const TileList* tl, int out_f64) {
    const TileList all{t.m_tile_sub, t.m_tile_row, t.m_tile_end, t.n_m_tiles};
    const TileList& L = tl ? *tl : all;
    if (L.n == 0) return;
    dim3 grid(L.n);
    const int nt = kFLThreads;
#define FL_ARGS t.subs, L.sub, L.row, L.end, k, Lambda, t.gmap, t.gmap_R
    if (precision == FETI_FP64) {
        k_flambda<FETI_FP64, double><<<grid, nt, 0, st>>>(FL_ARGS, Fsw, nullptr, (double*)Y, (double*)T);
    } else if (precision == FETI_FP32) {
        if (out_f64)
            k_flambda<FETI_FP32, double><<<grid, nt, 0, st>>>(FL_ARGS, Fsw, nullptr, (double*)Y, (double*)T);
        else
            k_flambda<FETI_FP32, float><<<grid, nt, 0, st>>>(FL_ARGS, Fsw, nullptr, (float*)Y, (float*)T);
    } else {
        if (out_f64)
            k_flambda<FETI_BF16X3, double><<<grid, nt, 0, st>>>(FL_ARGS, Fsw, Fsw_lo, (double*)Y, (double*)T);
        else
            k_flambda<FETI_BF16X3, float><<<grid, nt, 0, st>>>(FL_ARGS, Fsw, Fsw_lo, (float*)Y, (float*)T);
    }
#undef FL_ARGS
}

// ---------------------------------------------------------------------------------------
// FETI-DP corner coarse problem: t = add + sum_s B_c^sT T_s (one thread per entry, fixed
// summation order), then v = scale * Kbar_cc^{-1} t (workgroup = 32 rows x 16 columns with
// t staged through LDS in chunks of 64).
template <typename TT>
__global__ void k_coarse_t(int n_cg, int k, const TT* __restrict__ T, const double* __restrict__ add,
                           const int* __restrict__ cc_ptr, const int* __restrict__ cc_s, const int* __restrict__ cc_j,
                           const SubMeta* __restrict__ subs, double* __restrict__ t) {
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)n_cg * k) return;
    const int q = (int)(idx / k), c = (int)(idx % k);
    double val = add ? add[idx] : 0.0;
    for (int en = cc_ptr[q]; en < cc_ptr[q + 1]; ++en) val += (double)T[(subs[cc_s[en]].off_c + cc_j[en]) * k + c];
    t[idx] = val;
}

__global__ void __launch_bounds__(256) k_coarse_v(int n_cg, int k, const double* __restrict__ t,
                                                  const double* __restrict__ Kinv, double scale, double* __restrict__ v) {
    __shared__ double tc[64][17];
    const int p0 = blockIdx.x * 32, c0 = blockIdx.y * 16;
    const int tid = threadIdx.x;
    const int pr = tid >> 3, cg2 = (tid & 7) * 2;   // row p0+pr, columns c0+cg2, +1
    double acc0 = 0.0, acc1 = 0.0;
    const int p = p0 + pr;
    for (int q0 = 0; q0 < n_cg; q0 += 64) {
        for (int e = tid; e < 64 * 16; e += 256) {
            const int qq = e >> 4, c = e & 15;
            const int q = q0 + qq, col = c0 + c;
            tc[qq][c] = (q < n_cg && col < k) ? t[(long long)q * k + col] : 0.0;
        }
        __syncthreads();
        if (p < n_cg) {
            const int qn = min(64, n_cg - q0);
            const double* Kr = Kinv + (long long)p * n_cg + q0;
            for (int qq = 0; qq < qn; ++qq) {
                const double kv = Kr[qq];
                acc0 += kv * tc[qq][cg2];
                acc1 += kv * tc[qq][cg2 + 1];
            }
        }
        __syncthreads();
    }
    if (p < n_cg) {
        if (c0 + cg2 < k) v[(long long)p * k + c0 + cg2] = scale * acc0;
        if (c0 + cg2 + 1 < k) v[(long long)p * k + c0 + cg2 + 1] = scale * acc1;
    }
}

void launch_coarse(const DevTopo& t, int k, int ytype_f32, const void* T, const double* add, const double* Kinv,
                   double scale, double* v, double* tbuf, hipStream_t st) {
    if (t.n_cg == 0) return;
    const long long n = (long long)t.n_cg * k;
    if (ytype_f32)
        k_coarse_t<float><<<(int)((n + 255) / 256), 256, 0, st>>>(t.n_cg, k, (const float*)T, add, t.cc_ptr, t.cc_s,
                                                                  t.cc_j, t.subs, tbuf);
    else
        k_coarse_t<double><<<(int)((n + 255) / 256), 256, 0, st>>>(t.n_cg, k, (const double*)T, add, t.cc_ptr,
                                                                   t.cc_s, t.cc_j, t.subs, tbuf);
    k_coarse_v<<<dim3((t.n_cg + 31) / 32, (k + 15) / 16), 256, 0, st>>>(t.n_cg, k, tbuf, Kinv, scale, v);
}

// Y_s[j][c] += sum_q F_rc^s[j][q] v[cg(s,q)][c]  (the coarse correction folded into the local
// products before the scatter); workgroup = (subdomain, 64 interface rows), v_s in LDS.
template <typename TY>
__global__ void __launch_bounds__(256) k_fold_coarse(const SubMeta* __restrict__ subs, int k, const double* __restrict__ F64,
                                                     const int* __restrict__ c_glob, const double* __restrict__ v,
                                                     TY* __restrict__ Y) {
    __shared__ double vs[32][64];
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int j0 = blockIdx.x * 64;
    if (j0 >= M.n_b || M.n_c == 0) return;
    for (int e = threadIdx.x; e < M.n_c * 64; e += 256) {
        const int q = e >> 6, c = e & 63;
        vs[q][c] = c < k ? v[(long long)c_glob[M.off_c + q] * k + c] : 0.0;
    }
    __syncthreads();
    const int c = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (c >= k) return;
    for (int jj = wave; jj < 64; jj += 4) {
        const int j = j0 + jj;
        if (j >= M.n_b) break;
        const double* Fr = F64 + M.off_F + (long long)M.rowT * M.ldF + j;
        double acc = 0.0;
        for (int q = 0; q < M.n_c; ++q) acc += Fr[(long long)q * M.ldF] * vs[q][c];
        TY* y = Y + (M.off_b + j) * k + c;
        *y = (TY)((double)*y + acc);
    }
}

void launch_fold_coarse(const DevTopo& t, int k, int ytype_f32, const double* F64, const double* v, void* Y,
                        hipStream_t st) {
    if (t.n_cg == 0) return;
    dim3 grid((t.max_nb + 63) / 64, t.n_sub);
    if (ytype_f32)
        k_fold_coarse<float><<<grid, 256, 0, st>>>(t.subs, k, F64, t.c_glob, v, (float*)Y);
    else
        k_fold_coarse<double><<<grid, 256, 0, st>>>(t.subs, k, F64, t.c_glob, v, (double*)Y);
}

// Q[row][c] = sum over the row's (one or two) sides of sign * Y_s[j][c].
template <typename TY>
__global__ void k_scatter(int n_lambda, int k, const int* __restrict__ row_s, const int* __restrict__ row_j,
                          const int8_t* __restrict__ row_sg, const SubMeta* __restrict__ subs,
                          const TY* __restrict__ Y, double* __restrict__ Q) {
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)n_lambda * k) return;
    const int row = (int)(idx / k), c = (int)(idx % k);
    double val = 0.0;
    for (int t = 0; t < 2; ++t) {
        const int s = row_s[2 * row + t];
        if (s < 0) continue;
        val += row_sg[2 * row + t] * (double)Y[(subs[s].off_b + row_j[2 * row + t]) * k + c];
    }
    Q[idx] = val;
}

void launch_scatter(const DevTopo& t, int k, int ytype_f32, const void* Y, double* Q, hipStream_t st) {
    const long long n = (long long)t.n_lambda * k;
    if (n == 0) return;
    const int grid = (int)((n + 255) / 256);
    if (ytype_f32)
        k_scatter<float><<<grid, 256, 0, st>>>(t.n_lambda, k, t.row_s, t.row_j, t.row_sg, t.subs, (const float*)Y, Q);
    else
        k_scatter<double><<<grid, 256, 0, st>>>(t.n_lambda, k, t.row_s, t.row_j, t.row_sg, t.subs, (const double*)Y,
                                                Q);
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
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x * 256 >= M.n_b) return;
    for (int q = threadIdx.x; q < M.n_b; q += 256) {
        const long long g = M.off_b + q;
        double v = 0.0;
        for (int e = bg_ptr[g]; e < bg_ptr[g + 1]; ++e) v += bg_sg[e] * bg_w[e] * r[bg_row[e]];
        xs[q] = v;
    }
    __syncthreads();
    if (j >= M.n_b) return;
    // S~ is symmetric: y[j] = sum_q S~[q][j] x[q] reads column j, coalesced across threads
    const TP* Pc = P + M.off_P + j;
    double acc = 0.0;
#pragma unroll 8
    for (int q = 0; q < M.n_b; ++q) acc += (double)Pc[(long long)q * M.n_b] * xs[q];
    y[M.off_b + j] = acc;
}

void launch_precond_local(const DevTopo& t, int use_f32, const double* r, const double* bg_w, const double* P64,
                          const float* P32, double* y, hipStream_t st) {
    dim3 grid((t.max_nb + 255) / 256, t.n_sub);
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
