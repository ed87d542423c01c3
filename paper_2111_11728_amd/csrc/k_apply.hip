// Application of the dual operator F to a block of search directions (Sec. 2.1 Eq. 7,
// Sec. 2.2 Eq. 12 with u_c condensed), the preconditioner of Sec. 3.1 Eq. (13) and the
// TFETI projector.
//
// F * Lambda = sum_s B^s F_s B^sT Lambda runs in three launches:
//   1. k_flambda: one workgroup per (subdomain, row tile) gathers X_s = B^sT Lambda into LDS
//      (FP64, MFMA operand order, double-buffered 128-row chunks) and multiplies it by the
//      augmented operator A_s = [F_s; F_rc^sT] on the matrix cores. A_s streams from HBM in a
//      pre-swizzled layout (one coalesced 16-byte load per lane and MFMA step, prefetched one
//      step ahead). Row blocks of 16 rows run either in the reduced precision (two per
//      wavefront) or in FP64 (one per wavefront, same cost), both within one launch.
//   2. k_coarse (FETI-DP): t = sum_s B_c^sT F_rc^sT X_s, v = Kbar_cc^{-1} t.
//   3. k_scatter: owner-computes per lambda row, Q[row] = sum over the row's (one or two)
//      subdomains of sign * (Y_s[j] + F_rc^s[j,:] v_s); no atomics, bit-reproducible.
#include "kernels.hpp"

namespace feti {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kFLThreads = 64 * kFlWaves;
constexpr int kXC = 128;                         // rows of X_s per LDS chunk (two chunks in flight)
constexpr int kXPer = kXC * 64 / kFLThreads;     // gathered values per thread and chunk

__device__ inline __bf16 to_bf16(float x) {
    __hip_bfloat16 h = __float2bfloat16(x);
    return *reinterpret_cast<__bf16*>(&h);
}
__device__ inline float from_bf16(__bf16 x) { return __bfloat162float(*reinterpret_cast<__hip_bfloat16*>(&x)); }

// Gather of X_s rows [kc0, kc0 + kXC) through the fixed-width map gmap[q*R + t] =
// sign*(row+1) (0: unused slot). Value u of a thread is chunk row wave + 16 u, column lane:
// the row is uniform over the wavefront, so its map entries come through scalar loads and
// its Lambda row through one coalesced 512-byte load. gather_x only issues the loads of the
// first copy (nothing waits on them until the chunk is stored, after the next chunk's
// products); store_x applies the sign, adds further copies (rows shared by more than two
// subdomains) and writes the LDS chunk.
__device__ inline int fl_wave() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ inline void gather_x(const SubMeta& M, int kc0, int k, int R, const int* __restrict__ gmap,
                                const double* __restrict__ Lambda, double* g, int* gv) {
    const int wave = fl_wave();
    const int c = min((int)(threadIdx.x & 63), k - 1);
#pragma unroll
    for (int u = 0; u < kXPer; ++u) {
        const int j = kc0 + wave + 16 * u;
        gv[u] = j < M.n_b ? gmap[(M.off_b + j) * R] : 0;
    }
#pragma unroll
    for (int u = 0; u < kXPer; ++u) {
        const int r = gv[u] > 0 ? gv[u] - 1 : (gv[u] < 0 ? -gv[u] - 1 : 0);
        g[u] = Lambda[(long long)r * k + c];
    }
}

// LDS chunk layout (B operand of the 16x16x4 MFMAs): X[16 kq + 4 q + l/16][16 nb + l%16] is
// element (((kq*4 + nb)*2 + q/2)*64 + l)*2 + q%2: a lane's four operands of one 16-row step are
// two 16-byte pairs in two planes, so every 16-byte read has a 16-byte lane stride (no bank
// conflicts). Chunk row wave + 16 u has kq = u, q = wave/4, l/16 = wave%4.
__device__ __forceinline__ int x_index(int kq, int nb, int l, int q) {
    return (((kq * 4 + nb) * 2 + (q >> 1)) * 64 + l) * 2 + (q & 1);
}
__device__ __forceinline__ v4d ld_x(const double* Xb, int kq, int nb, int lane) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 lo = *reinterpret_cast<const v2*>(Xb + x_index(kq, nb, lane, 0));
    const v2 hi = *reinterpret_cast<const v2*>(Xb + x_index(kq, nb, lane, 2));
    return v4d{lo[0], lo[1], hi[0], hi[1]};
}
__device__ inline void store_x(double* Xb, const SubMeta& M, int kc0, int k, int R, const int* __restrict__ gmap,
                               const double* __restrict__ Lambda, const double* g, const int* gv) {
    const int wave = fl_wave();
    const int lane = threadIdx.x & 63;
    const int c = min(lane, k - 1);
#pragma unroll
    for (int u = 0; u < kXPer; ++u) {
        double v = gv[u] > 0 ? g[u] : (gv[u] < 0 ? -g[u] : 0.0);
        if (R > 1 && gv[u] != 0) {
            const int* gm = gmap + (M.off_b + kc0 + wave + 16 * u) * R;
            for (int t = 1; t < R; ++t) {
                const int e = gm[t];
                if (e > 0) v += Lambda[(long long)(e - 1) * k + c];
                else if (e < 0) v -= Lambda[(long long)(-e - 1) * k + c];
            }
        }
        if (lane >= k) v = 0.0;
        Xb[x_index(u, lane >> 4, (wave & 3) * 16 + (lane & 15), wave >> 2)] = v;
    }
}

__device__ inline void split_bf16(double x, __bf16& hi, __bf16& lo) {
    const float f = (float)x;
    hi = to_bf16(f);
    lo = to_bf16(f - from_bf16(hi));
}

template <typename Out>
__device__ inline void store_block(const SubMeta& M, int row0, int lane, int k, int nbk, bool f64_layout, bool storeT,
                                   const float* accf, const double* accd, Out* __restrict__ Y, Out* __restrict__ T) {
    // D layout of the 16x16 blocks: column lane%16; rows 4*(lane/16)+v (FP32 accumulators)
    // or lane/16 + 4*v (FP64 accumulators)
    for (int nb = 0; nb < nbk; ++nb) {
        const int col = nb * 16 + (lane & 15);
        if (col >= k) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + (f64_layout ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
            const Out val = f64_layout ? (Out)accd[nb * 4 + v] : (Out)accf[nb * 4 + v];
            if (row < M.n_b)
                Y[(M.off_b + row) * k + col] = val;
            else if (storeT && row >= M.rowT && row < M.rowT + M.n_c)
                T[(M.off_c + row - M.rowT) * k + col] = val;
        }
    }
}

// Each wavefront runs the whole chunk loop for its role; every role gathers its share of
// the X_s chunks and meets the same nch + 1 workgroup barriers, so the roles' register
// states never overlap.
struct FlCtx {
    const SubMeta& M;
    int k, R, lane;
    const int* gmap;
    const double* Lambda;
    double* Xs;   // two chunk buffers of kXC*64 doubles
};

__device__ inline int fl_nch(const SubMeta& M) { return (M.ldF + kXC - 1) / kXC; }

template <typename Body>
__device__ __forceinline__ void fl_chunks(const FlCtx& C, Body body) {
    double g[kXPer];
    int gv[kXPer];
    gather_x(C.M, 0, C.k, C.R, C.gmap, C.Lambda, g, gv);
    store_x(C.Xs, C.M, 0, C.k, C.R, C.gmap, C.Lambda, g, gv);
    __syncthreads();
    const int nch = fl_nch(C.M);
    for (int ch = 0; ch < nch; ++ch) {
        const int kc0 = ch * kXC;
        if (ch + 1 < nch) gather_x(C.M, kc0 + kXC, C.k, C.R, C.gmap, C.Lambda, g, gv);
        body(C.Xs + (ch & 1) * (kXC * 64), kc0, min(kXC, C.M.ldF - kc0));
        if (ch + 1 < nch) store_x(C.Xs + ((ch + 1) & 1) * (kXC * 64), C.M, kc0 + kXC, C.k, C.R, C.gmap, C.Lambda, g, gv);
        __syncthreads();
    }
}

template <int NB, typename Out>
__device__ __forceinline__ void fl_fp32(const FlCtx& C, const float* __restrict__ Ared, int rb0, int rb1, bool two,
                                        bool storeT, Out* __restrict__ Y, Out* __restrict__ T) {
    const SubMeta& M = C.M;
    const int lane = C.lane, KQ = M.ldF >> 4;
    const float* A = Ared + M.off_Fsw + lane * 4;
    const float* p0 = A + (long long)rb0 * KQ * 256;
    const float* p1 = A + (long long)rb1 * KQ * 256;
    v4f acc0[NB], acc1[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc0[nb] = acc1[nb] = v4f{0.f, 0.f, 0.f, 0.f};
    v4f n0 = *reinterpret_cast<const v4f*>(p0), n1 = *reinterpret_cast<const v4f*>(p1);
    fl_chunks(C, [&](const double* Xb, int kc0, int kcn) {
        for (int kql = 0; kql < (kcn >> 4); ++kql) {
            const int gkq = (kc0 >> 4) + kql;
            const v4f a0 = n0, a1 = n1;
            if (gkq + 1 < KQ) {
                n0 = *reinterpret_cast<const v4f*>(p0 + (gkq + 1) * 256);
                n1 = *reinterpret_cast<const v4f*>(p1 + (gkq + 1) * 256);
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const v4d xv = ld_x(Xb, kql, nb, lane);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float b = (float)xv[q];
                    acc0[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[q], b, acc0[nb], 0, 0, 0);
                    acc1[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[q], b, acc1[nb], 0, 0, 0);
                }
            }
        }
    });
    float f[4 * NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) f[nb * 4 + v] = acc0[nb][v];
    store_block<Out>(M, 16 * rb0, lane, C.k, NB, false, storeT, f, nullptr, Y, T);
    if (two) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) f[nb * 4 + v] = acc1[nb][v];
        store_block<Out>(M, 16 * rb1, lane, C.k, NB, false, storeT, f, nullptr, Y, T);
    }
}

template <int NB, typename Out>
__device__ __forceinline__ void fl_bf16(const FlCtx& C, const __bf16* __restrict__ Ahi, const __bf16* __restrict__ Alo,
                                        int rb0, int rb1, bool two, bool storeT, Out* __restrict__ Y, Out* __restrict__ T) {
    const SubMeta& M = C.M;
    const int lane = C.lane, KB = M.ldF >> 5;
    const v8bf* H = reinterpret_cast<const v8bf*>(Ahi) + (M.off_Fsw >> 3) + lane;
    const v8bf* L = reinterpret_cast<const v8bf*>(Alo) + (M.off_Fsw >> 3) + lane;
    const v8bf* h0p = H + (long long)rb0 * KB * 64;
    const v8bf* h1p = H + (long long)rb1 * KB * 64;
    const v8bf* l0p = L + (long long)rb0 * KB * 64;
    const v8bf* l1p = L + (long long)rb1 * KB * 64;
    v4f acc0[NB], acc1[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc0[nb] = acc1[nb] = v4f{0.f, 0.f, 0.f, 0.f};
    v8bf nh0 = *h0p, nh1 = *h1p, nl0 = *l0p, nl1 = *l1p;
    fl_chunks(C, [&](const double* Xb, int kc0, int kcn) {
        for (int kbl = 0; kbl < (kcn >> 5); ++kbl) {
            const int gkb = (kc0 >> 5) + kbl;
            const v8bf h0 = nh0, h1 = nh1, l0 = nl0, l1 = nl1;
            if (gkb + 1 < KB) {
                nh0 = h0p[(gkb + 1) * 64];
                nh1 = h1p[(gkb + 1) * 64];
                nl0 = l0p[(gkb + 1) * 64];
                nl1 = l1p[(gkb + 1) * 64];
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                // lane operand e = 4h + q is X row 32 kb + 16 h + 4 q + lane/16 (the A layout
                // uses the same permutation of the contraction index)
                const v4d x0 = ld_x(Xb, 2 * kbl, nb, lane);
                const v4d x1 = ld_x(Xb, 2 * kbl + 1, nb, lane);
                v8bf bh, bl;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    __bf16 hi, lo;
                    split_bf16(x0[q], hi, lo);
                    bh[q] = hi;
                    bl[q] = lo;
                    split_bf16(x1[q], hi, lo);
                    bh[4 + q] = hi;
                    bl[4 + q] = lo;
                }
                acc0[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h0, bh, acc0[nb], 0, 0, 0);
                acc0[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h0, bl, acc0[nb], 0, 0, 0);
                acc0[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l0, bh, acc0[nb], 0, 0, 0);
                acc1[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h1, bh, acc1[nb], 0, 0, 0);
                acc1[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h1, bl, acc1[nb], 0, 0, 0);
                acc1[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l1, bh, acc1[nb], 0, 0, 0);
            }
        }
    });
    float f[4 * NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) f[nb * 4 + v] = acc0[nb][v];
    store_block<Out>(M, 16 * rb0, lane, C.k, NB, false, storeT, f, nullptr, Y, T);
    if (two) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) f[nb * 4 + v] = acc1[nb][v];
        store_block<Out>(M, 16 * rb1, lane, C.k, NB, false, storeT, f, nullptr, Y, T);
    }
}

template <int NB, typename Out>
__device__ __forceinline__ void fl_fp64(const FlCtx& C, const double* __restrict__ A64, int rb0, Out* __restrict__ Y,
                                        Out* __restrict__ T) {
    const SubMeta& M = C.M;
    const int lane = C.lane, KQ = M.ldF >> 4;
    const double* p = A64 + M.off_Fsw + (long long)rb0 * KQ * 256 + lane * 4;
    v4d acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = v4d{0.0, 0.0, 0.0, 0.0};
    v4d n = *reinterpret_cast<const v4d*>(p);
    fl_chunks(C, [&](const double* Xb, int kc0, int kcn) {
        for (int kql = 0; kql < (kcn >> 4); ++kql) {
            const int gkq = (kc0 >> 4) + kql;
            const v4d a = n;
            if (gkq + 1 < KQ) n = *reinterpret_cast<const v4d*>(p + (gkq + 1) * 256);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const v4d xv = ld_x(Xb, kql, nb, lane);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], xv[q], acc[nb], 0, 0, 0);
            }
        }
    });
    double d[4 * NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) d[nb * 4 + v] = acc[nb][v];
    store_block<Out>(M, 16 * rb0, lane, C.k, NB, true, true, nullptr, d, Y, T);
}

// Up to four FP64 row blocks with the contraction split four ways: wavefront w takes row
// block d0 + w/4 and, in every X_s chunk, the 16-column steps 8ch + (w%4) + 4j (j = 0, 1), whose
// operands it loads one chunk ahead; the four partial blocks of each row block then meet in
// LDS and are summed in slice order (deterministic).
template <int NB, typename Out>
__device__ __forceinline__ void fl_fp64_splitk(const FlCtx& C, const double* __restrict__ A64, int d0, int n_d,
                                               Out* __restrict__ Y, Out* __restrict__ T) {
    constexpr int S = 4;
    static_assert(kXC == 128, "two steps per slice and chunk");
    const SubMeta& M = C.M;
    const int lane = C.lane, wave = fl_wave(), KQ = M.ldF >> 4;
    const int ri = wave / S, sl = wave % S;
    const bool act = ri < n_d;
    const double* p = A64 + M.off_Fsw + (long long)(d0 + (act ? ri : 0)) * KQ * 256 + lane * 4;
    auto ld = [&](int ch, v4d* a) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int kq = 8 * ch + sl + 4 * j;
            a[j] = (act && kq < KQ) ? *reinterpret_cast<const v4d*>(p + kq * 256) : v4d{0.0, 0.0, 0.0, 0.0};
        }
    };
    v4d acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = v4d{0.0, 0.0, 0.0, 0.0};
    v4d pre[2];
    ld(0, pre);
    int ch = 0;
    fl_chunks(C, [&](const double* Xb, int kc0, int kcn) {
        const v4d cur[2] = {pre[0], pre[1]};
        ld(ch + 1, pre);
        if (act) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int kql = sl + 4 * j;
                if (kql < (kcn >> 4)) {
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        const v4d xv = ld_x(Xb, kql, nb, lane);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[j][q], xv[q], acc[nb], 0, 0, 0);
                    }
                }
            }
        }
        ++ch;
    });
    // partials: Xs[(w * 4 NB + nb * 4 + v) * 64 + lane] (the chunk buffers are free after the last barrier)
    double* P = C.Xs;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) P[(wave * 4 * NB + nb * 4 + v) * 64 + lane] = acc[nb][v];
    __syncthreads();
    for (int e = threadIdx.x; e < n_d * 4 * NB * 64; e += kFLThreads) {
        const int r = e / (4 * NB * 64), el = e - r * (4 * NB * 64);
        double sum = 0.0;
        for (int w = r * S; w < (r + 1) * S; ++w) sum += P[w * 4 * NB * 64 + el];
        const int nbv = el >> 6, l = el & 63, nb = nbv >> 2, v = nbv & 3;
        const int row = 16 * (d0 + r) + (l >> 4) + 4 * v, col = nb * 16 + (l & 15);
        if (col < C.k) {
            if (row < M.n_b)
                Y[(M.off_b + row) * C.k + col] = (Out)sum;
            else if (row >= M.rowT && row < M.rowT + M.n_c)
                T[(M.off_c + row - M.rowT) * C.k + col] = (Out)sum;
        }
    }
}

// One reduced-precision row block and one FP64 row block in the same wavefront (a tile whose
// reduced row-block count is odd gives its last reduced wavefront the first FP64 block; both
// together cost one FP32 pair).
template <int P, int NB, typename Out>
__device__ __forceinline__ void fl_mixed(const FlCtx& C, const void* __restrict__ Ared_, const void* __restrict__ Ared_lo_,
                                         const double* __restrict__ A64, int rbr, int rbd, Out* __restrict__ Y,
                                         Out* __restrict__ T) {
    const SubMeta& M = C.M;
    const int lane = C.lane, KQ = M.ldF >> 4, KB = M.ldF >> 5;
    v4f accr[NB];
    v4d accd[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        accr[nb] = v4f{0.f, 0.f, 0.f, 0.f};
        accd[nb] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    const double* pd = A64 + M.off_Fsw + (long long)rbd * KQ * 256 + lane * 4;
    fl_chunks(C, [&](const double* Xb, int kc0, int kcn) {
        if constexpr (P == FETI_FP32) {
            const float* pf = reinterpret_cast<const float*>(Ared_) + M.off_Fsw + (long long)rbr * KQ * 256 + lane * 4;
            for (int kql = 0; kql < (kcn >> 4); ++kql) {
                const int gkq = (kc0 >> 4) + kql;
                const v4f af = *reinterpret_cast<const v4f*>(pf + gkq * 256);
                const v4d ad = *reinterpret_cast<const v4d*>(pd + gkq * 256);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const v4d xv = ld_x(Xb, kql, nb, lane);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        accr[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[q], (float)xv[q], accr[nb], 0, 0, 0);
                        accd[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad[q], xv[q], accd[nb], 0, 0, 0);
                    }
                }
            }
        } else {
            const v8bf* H = reinterpret_cast<const v8bf*>(Ared_) + (M.off_Fsw >> 3) + lane + (long long)rbr * KB * 64;
            const v8bf* L = reinterpret_cast<const v8bf*>(Ared_lo_) + (M.off_Fsw >> 3) + lane + (long long)rbr * KB * 64;
            for (int kbl = 0; kbl < (kcn >> 5); ++kbl) {
                const int gkb = (kc0 >> 5) + kbl;
                const v8bf h = H[gkb * 64], l = L[gkb * 64];
                const v4d ad0 = *reinterpret_cast<const v4d*>(pd + (2 * gkb) * 256);
                const v4d ad1 = *reinterpret_cast<const v4d*>(pd + (2 * gkb + 1) * 256);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const v4d x0 = ld_x(Xb, 2 * kbl, nb, lane);
                    const v4d x1 = ld_x(Xb, 2 * kbl + 1, nb, lane);
                    v8bf bh, bl;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        __bf16 hi, lo;
                        split_bf16(x0[q], hi, lo);
                        bh[q] = hi;
                        bl[q] = lo;
                        split_bf16(x1[q], hi, lo);
                        bh[4 + q] = hi;
                        bl[4 + q] = lo;
                    }
                    accr[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bh, accr[nb], 0, 0, 0);
                    accr[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bl, accr[nb], 0, 0, 0);
                    accr[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l, bh, accr[nb], 0, 0, 0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        accd[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad0[q], x0[q], accd[nb], 0, 0, 0);
                        accd[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ad1[q], x1[q], accd[nb], 0, 0, 0);
                    }
                }
            }
        }
    });
    float f[4 * NB];
    double d[4 * NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            f[nb * 4 + v] = accr[nb][v];
            d[nb * 4 + v] = accd[nb][v];
        }
    store_block<Out>(M, 16 * rbr, lane, C.k, NB, false, false, f, nullptr, Y, T);
    store_block<Out>(M, 16 * rbd, lane, C.k, NB, true, true, nullptr, d, Y, T);
}

// P: precision of the reduced row blocks (FETI_FP64: none); NB: 16-column blocks of the
// direction block computed (1 for k <= 16, else 4).
template <int P, int NB, typename Out>
__global__ void __launch_bounds__(kFLThreads) k_flambda(const SubMeta* __restrict__ subs, const FlTile* __restrict__ tiles,
                                                        int k, const double* __restrict__ Lambda,
                                                        const int* __restrict__ gmap, int R,
                                                        const void* __restrict__ Ared_, const void* __restrict__ Ared_lo_,
                                                        const double* __restrict__ A64,
                                                        Out* __restrict__ Y, Out* __restrict__ T) {
    __shared__ __attribute__((aligned(16))) double Xs[2 * kXC * 64];
    const FlTile tl = tiles[blockIdx.x];
    if (tl.s < 0) return;
    const SubMeta M = subs[tl.s];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const FlCtx C{M, k, R, lane, gmap, Lambda, Xs};
    if (tl.flags & kFlSplitK) {
        fl_fp64_splitk<NB, Out>(C, A64, tl.d0, tl.n_d, Y, T);
        return;
    }
    // wavefront role (uniform): two reduced row blocks; one reduced and one FP64 row block (the
    // last reduced wavefront of an odd count, when FP64 blocks follow); one FP64 row block; or
    // gather only
    const int nw_red = (tl.n_red + 1) >> 1;
    const int mixed = P != FETI_FP64 && (tl.n_red & 1) && tl.n_d > 0;
    if (P != FETI_FP64 && wave < nw_red) {
        const int rb0 = tl.red0 + 2 * wave;
        const bool two = 2 * wave + 1 < tl.n_red;
        const int rb1 = two ? rb0 + 1 : rb0;
        const bool storeT = !(tl.flags & kFlNoT);
        if constexpr (P != FETI_FP64) {
            if (!two && mixed) {
                fl_mixed<P, NB, Out>(C, Ared_, Ared_lo_, A64, rb0, tl.d0, Y, T);
                return;
            }
        }
        if constexpr (P == FETI_FP32)
            fl_fp32<NB, Out>(C, reinterpret_cast<const float*>(Ared_), rb0, rb1, two, storeT, Y, T);
        else if constexpr (P == FETI_BF16X3)
            fl_bf16<NB, Out>(C, reinterpret_cast<const __bf16*>(Ared_), reinterpret_cast<const __bf16*>(Ared_lo_), rb0,
                             rb1, two, storeT, Y, T);
    } else if (wave >= nw_red && wave - nw_red < tl.n_d - mixed) {
        fl_fp64<NB, Out>(C, A64, tl.d0 + mixed + wave - nw_red, Y, T);
    } else {
        fl_chunks(C, [](const double*, int, int) {});
    }
}

template <int P, typename Out>
void launch_fl(const DevTopo& t, const FlTiles& L, int k, const double* Lambda, const void* Ared, const void* Ared_lo,
               const double* A64, Out* Y, Out* T, hipStream_t st) {
    if (k <= 16)
        k_flambda<P, 1, Out><<<L.n, kFLThreads, 0, st>>>(t.subs, L.t, k, Lambda, t.gmap, t.gmap_R, Ared, Ared_lo, A64, Y, T);
    else
        k_flambda<P, 4, Out><<<L.n, kFLThreads, 0, st>>>(t.subs, L.t, k, Lambda, t.gmap, t.gmap_R, Ared, Ared_lo, A64, Y, T);
}

void launch_flambda(const DevTopo& t, int precision, int k, const double* Lambda, const void* Ared, const void* Ared_lo,
                    const double* A64, void* Y, void* T, hipStream_t st, const FlTiles* tl, int out_f64) {
    if (k < 1 || k > 64) throw std::invalid_argument("F*Lambda takes 1..64 directions");
    if (t.n_lambda < 1) throw std::invalid_argument("F*Lambda without Lagrange multipliers");
    const FlTiles& L = tl ? *tl : (precision == FETI_FP64 ? t.fl64 : t.flred);
    if (L.n == 0) return;
    if (precision == FETI_FP64) {
        launch_fl<FETI_FP64, double>(t, L, k, Lambda, nullptr, nullptr, A64, (double*)Y, (double*)T, st);
    } else if (precision == FETI_FP32) {
        if (out_f64)
            launch_fl<FETI_FP32, double>(t, L, k, Lambda, Ared, nullptr, A64, (double*)Y, (double*)T, st);
        else
            launch_fl<FETI_FP32, float>(t, L, k, Lambda, Ared, nullptr, A64, (float*)Y, (float*)T, st);
    } else {
        if (out_f64)
            launch_fl<FETI_BF16X3, double>(t, L, k, Lambda, Ared, Ared_lo, A64, (double*)Y, (double*)T, st);
        else
            launch_fl<FETI_BF16X3, float>(t, L, k, Lambda, Ared, Ared_lo, A64, (float*)Y, (float*)T, st);
    }
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

// v = scale * Kinv t (n_cg x n_cg by n_cg x k, k <= 64) on the FP64 matrix cores: workgroup =
// 16 rows and 16 columns (16 blockIdx.y .. + 15) of v. Step Q contracts q = 16Q + 4g + s, so
// lane (m, g) reads Kinv[p0 + m][16Q + 4g .. +3] (one 32-byte load) and t[16Q + 4g + s][col].
__global__ void __launch_bounds__(256) k_coarse_v(const CoarseTile* __restrict__ tiles,
                                                  const CoarseBlk* __restrict__ blks, int k, const double* __restrict__ tg,
                                                  const double* __restrict__ Kg, double scale, double* __restrict__ vg) {
    // workgroup: 16 rows of v inside one design's block (v_B = Kbar_B^{-1} t_B) and one 16-column
    // group cg; wavefront ks takes the 16-wide contraction slices Q = ks (mod 4), three slices of
    // loads in flight; the four partial tiles are summed in LDS in a fixed order
    typedef double v4 __attribute__((ext_vector_type(4)));
    __shared__ double red[4][16][16];
    const CoarseTile T = tiles[blockIdx.x];
    const CoarseBlk B = blks[T.blk];
    const int n_cg = B.n;
    const double* __restrict__ Kinv = Kg + B.off;
    const double* __restrict__ t = tg + (long long)B.cg0 * k;
    double* __restrict__ v = vg + (long long)B.cg0 * k;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, m = lane & 15, g = lane >> 4;
    const int cg = blockIdx.y, ks = wave;
    const int p0 = T.r0, col = 16 * cg + m;
    const int prow = p0 + m;
    const int nQ = (n_cg + 15) >> 4;
    const bool vec = (n_cg & 3) == 0;
    auto ld = [&](int Q, double (&a)[4], double (&bq)[4]) {
        const int q0 = 16 * Q + 4 * g;
        if (Q < nQ && vec && prow < n_cg && q0 + 3 < n_cg) {
            const v4 av = *reinterpret_cast<const v4*>(Kinv + (long long)prow * n_cg + q0);
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) a[s2] = av[s2];
        } else {
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2)
                a[s2] = (Q < nQ && prow < n_cg && q0 + s2 < n_cg) ? Kinv[(long long)prow * n_cg + q0 + s2] : 0.0;
        }
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2)
            bq[s2] = (Q < nQ && q0 + s2 < n_cg && col < k) ? t[(long long)(q0 + s2) * k + col] : 0.0;
    };
    constexpr int R = 3;
    double ar[R][4], br[R][4];
#pragma unroll
    for (int d = 0; d < R; ++d) ld(ks + 4 * d, ar[d], br[d]);
    v4 acc = v4{0.0, 0.0, 0.0, 0.0};
    for (int Q = ks; Q < nQ; Q += 4 * R) {
#pragma unroll
        for (int d = 0; d < R; ++d) {
            if (Q + 4 * d < nQ) {
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[d][s2], br[d][s2], acc, 0, 0, 0);
                ld(Q + 4 * d + 4 * R, ar[d], br[d]);
            }
        }
    }
    // D layout: rows g + 4 j, column m
#pragma unroll
    for (int j = 0; j < 4; ++j) red[ks][g + 4 * j][m] = acc[j];
    __syncthreads();
    if (ks == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = g + 4 * j, p = p0 + r;
            if (p < n_cg && col < k)
                v[(long long)p * k + col] = scale * (((red[0][r][m] + red[1][r][m]) + red[2][r][m]) + red[3][r][m]);
        }
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
    k_coarse_v<<<dim3(t.n_ctiles, (k + 15) / 16), 256, 0, st>>>(t.ctiles, t.cblk, k, tbuf, Kinv, scale, v);
}

// Y_s[j][c] += sum_q F_rc^s[j][q] v[cg(s,q)][c]  (the coarse correction folded into the local
// products before the scatter); workgroup = (subdomain, 64 interface rows), v_s in LDS.
template <typename TY>
__global__ void __launch_bounds__(256) k_fold_coarse(const SubMeta* __restrict__ subs, int k, const double* __restrict__ F64,
                                                     const int* __restrict__ c_glob, const double* __restrict__ v,
                                                     TY* __restrict__ Y) {
    __shared__ double vs[32][64];
    __shared__ double Fs[32][64];   // Fs[q][jj] = F_rc^T[q][j0 + jj]
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int j0 = blockIdx.x * 64;
    if (j0 >= M.n_b || M.n_c == 0) return;
    for (int e = threadIdx.x; e < M.n_c * 64; e += 256) {
        const int q = e >> 6, c = e & 63;
        vs[q][c] = c < k ? v[(long long)c_glob[M.off_c + q] * k + c] : 0.0;
        Fs[q][c] = j0 + c < M.n_b ? F64[M.off_F + (long long)(M.rowT + q) * M.ldF + j0 + c] : 0.0;
    }
    __syncthreads();
    const int c = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (c >= k) return;
    const int nj = min(64, M.n_b - j0);
    TY y[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int jj = wave + 4 * i;
        y[i] = jj < nj ? Y[(M.off_b + j0 + jj) * k + c] : (TY)0;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int jj = wave + 4 * i;
        double acc = 0.0;
        for (int q = 0; q < M.n_c; ++q) acc += Fs[q][jj] * vs[q][c];
        if (jj < nj) Y[(M.off_b + j0 + jj) * k + c] = (TY)((double)y[i] + acc);
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
__global__ void k_scatter(int n_lambda, int k, const long long* __restrict__ row_yo, const int8_t* __restrict__ row_sg,
                          const TY* __restrict__ Y, double* __restrict__ Q) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_lambda * k) return;
    const int row = k == 64 ? idx >> 6 : idx / k, c = idx - row * k;
    double val = 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const long long yo = row_yo[2 * row + t];
        if (yo >= 0) val += row_sg[2 * row + t] * (double)Y[yo * k + c];
    }
    Q[idx] = val;
}

void launch_scatter(const DevTopo& t, int k, int ytype_f32, const void* Y, double* Q, hipStream_t st) {
    const long long n = (long long)t.n_lambda * k;
    if (n == 0) return;
    const int grid = (int)((n + 255) / 256);
    if (ytype_f32)
        k_scatter<float><<<grid, 256, 0, st>>>(t.n_lambda, k, t.row_yo, t.row_sg, (const float*)Y, Q);
    else
        k_scatter<double><<<grid, 256, 0, st>>>(t.n_lambda, k, t.row_yo, t.row_sg, (const double*)Y, Q);
}

// Entries of B_r F_rc B_c (Sec. 2.2, Eq. 12) per lambda row: side t of the row (subdomain s,
// interface position j, sign) contributes sign * F_rc^s[j][q] for each of the subdomain's corner
// DOFs q, read from the F_rc^T rows of the augmented operator. One thread per row.
// (fr_val2, when given: the same values at the row's position ipos[r] in the pair-grouped order)
__global__ void k_fold_rows(int n_lambda, int W, const int* __restrict__ row_s, const int* __restrict__ row_j,
                            const int8_t* __restrict__ row_sg, const SubMeta* __restrict__ subs,
                            const double* __restrict__ F64, double* __restrict__ fr_val,
                            const int* __restrict__ ipos, double* __restrict__ fr_val2) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_lambda) return;
    const long long r2 = fr_val2 ? (long long)ipos[r] * W : 0;
    int e = 0;
    for (int t = 0; t < 2; ++t) {
        const int s = row_s[2 * r + t];
        if (s < 0) continue;
        const SubMeta M = subs[s];
        const int j = row_j[2 * r + t];
        const double sg = (double)row_sg[2 * r + t];
        for (int q = 0; q < M.n_c && e < W; ++q, ++e) {
            const double val = sg * F64[M.off_F + (long long)(M.rowT + q) * M.ldF + j];
            fr_val[(long long)r * W + e] = val;
            if (fr_val2) fr_val2[r2 + e] = val;
        }
    }
}

void launch_fold_rows(const DevTopo& t, const double* F64, hipStream_t st) {
    if (t.n_cg == 0 || t.n_lambda == 0 || t.fr_w == 0) return;
    k_fold_rows<<<(t.n_lambda + 255) / 256, 256, 0, st>>>(t.n_lambda, t.fr_w, t.row_s, t.row_j, t.row_sg, t.subs,
                                                          F64, t.fr_val, t.pr_ipos, t.n_pairs ? t.pr_fval : nullptr);
}

// Q[row][c] = sum over the row's sides of sign * Y_s[j][c] + sum_e fr_val[row][e] v[fr_col[row][e]][c]:
// the owner-computes scatter and the coarse fold Y_s += F_rc^s B_c^s v in one pass, so the local
// products are read once and never rewritten. With k = 64 a wavefront is one row: its map entries
// are wavefront-uniform scalar loads, v rows are 512-byte lines (L2-resident: n_cg x k).
template <typename TY>
__global__ void __launch_bounds__(256) k_scatter_fold(int n_lambda, int k, int W, const long long* __restrict__ row_yo,
                                                      const int8_t* __restrict__ row_sg, const TY* __restrict__ Y,
                                                      const int* __restrict__ fr_n, const int* __restrict__ fr_col,
                                                      const double* __restrict__ fr_val, const double* __restrict__ v,
                                                      double* __restrict__ Q) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_lambda * k) return;
    int row = k == 64 ? idx >> 6 : idx / k;
    if (k == 64) row = __builtin_amdgcn_readfirstlane(row);
    const int c = idx - row * k;
    double val = 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const long long yo = row_yo[2 * row + t];
        if (yo >= 0) val += row_sg[2 * row + t] * (double)Y[yo * k + c];
    }
    const int ne = fr_n[row];
    const int* __restrict__ fc = fr_col + (long long)row * W;
    const double* __restrict__ fv = fr_val + (long long)row * W;
    double acc0 = 0.0, acc1 = 0.0;
    int e = 0;
    for (; e + 1 < ne; e += 2) {
        acc0 = fma(fv[e], v[(long long)fc[e] * k + c], acc0);
        acc1 = fma(fv[e + 1], v[(long long)fc[e + 1] * k + c], acc1);
    }
    if (e < ne) acc0 = fma(fv[e], v[(long long)fc[e] * k + c], acc0);
    Q[idx] = val + (acc0 + acc1);
}

// The same per pair of subdomains, for blocks of 32 or more columns: workgroup g stages the
// coarse solution rows of its group's corner union (at most 64 x 64) in LDS once; its sixteen
// wavefronts take the group's rows kFoldRows at a time each (wavefront w: rows w, w + 16, ...), a
// lane per column. Every per-row array is stored in the group order, so a row's loads depend on
// nothing but its position, and a row's fold entries (at most 64) come in with one vector load per
// table, lane e holding entry e, and are broadcast by readlane: no memory load waits inside the
// fold loop. The first pass's table and local-product loads are issued before the staging of the
// coarse rows and its barrier (the only one, met by every wavefront), so the whole group's reads
// are in flight together.
__device__ __forceinline__ double bcast_lane(double v, int e) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), e);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), e);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One pass's loads: rows base .. base + kFoldRows - 1 of the group. Their records are contiguous:
// one scalar load from min(base, i1 - 1), which stays inside the table (it carries kFoldRows
// padding records after its last row). Rows at or past i1 are masked (no fold entries, both
// sides absent, no store), and an absent side reads local product row 0 and adds nothing, so the
// loads carry no branches.
// side[r] = sign_0 Y_0[c] + sign_1 Y_1[c] over the row's sides; fp/fv: the fold entry of lane c.
typedef int fold_rec_t __attribute__((ext_vector_type(4 * kFoldRows)));
template <typename TY>
__device__ __forceinline__ void fold_rows_load(int base, int i1, int k, int W, int c, const int4* __restrict__ pr_rec,
                                               const int* __restrict__ pr_fpos, const double* __restrict__ pr_fval,
                                               const TY* __restrict__ Y, int4 (&rec)[kFoldRows],
                                               double (&side)[kFoldRows], int (&fp)[kFoldRows],
                                               double (&fv)[kFoldRows]) {
    const int lb = min(base, i1 - 1);
    const fold_rec_t all = *reinterpret_cast<const fold_rec_t*>(pr_rec + lb);
#pragma unroll
    for (int r = 0; r < kFoldRows; ++r) {
        const bool in = base + r < i1 && lb == base;   // lb < base only when base >= i1
        rec[r] = in ? int4{all[4 * r], all[4 * r + 1], all[4 * r + 2], all[4 * r + 3]} : int4{-1, -1, 0, 0};
    }
    const int cc = c < k ? c : 0;
#pragma unroll
    for (int r = 0; r < kFoldRows; ++r) {
        const bool e = c < (rec[r].z >> 2);
        const long long ce = e ? (long long)(base + r) * W + c : 0;
        const int p = pr_fpos[ce];
        const double v = pr_fval[ce];
        fp[r] = e ? p : 0;
        fv[r] = e ? v : 0.0;
        const double a0 = (double)Y[(long long)max(rec[r].x, 0) * k + cc];
        const double a1 = (double)Y[(long long)max(rec[r].y, 0) * k + cc];
        const double s0 = (rec[r].z & 1) ? -1.0 : 1.0, s1 = (rec[r].z & 2) ? -1.0 : 1.0;
        double sd = 0.0;
        sd += rec[r].x >= 0 ? s0 * a0 : 0.0;
        sd += rec[r].y >= 0 ? s1 * a1 : 0.0;
        side[r] = sd;
    }
}

// The fold sums and the stores of one pass.
__device__ __forceinline__ void fold_rows_store(int base, int i1, int k, int c, const double (*vs)[64],
                                                const int4 (&rec)[kFoldRows], const double (&side)[kFoldRows],
                                                const int (&fp)[kFoldRows], const double (&fv)[kFoldRows],
                                                double* __restrict__ Q) {
#pragma unroll
    for (int r = 0; r < kFoldRows; ++r) {
        double a = 0.0;
        const int ne = rec[r].z >> 2;
        for (int e = 0; e < ne; ++e) a = fma(bcast_lane(fv[r], e), vs[__builtin_amdgcn_readlane(fp[r], e)][c], a);
        if (base + r < i1 && c < k) Q[(long long)rec[r].w * k + c] = side[r] + a;
    }
}

template <typename TY>
__global__ void __launch_bounds__(1024) k_scatter_fold_pair(int k, int W, const int* __restrict__ pr_ptr,
                                                            const int4* __restrict__ pr_rec,
                                                            const int* __restrict__ pr_fpos,
                                                            const double* __restrict__ pr_fval,
                                                            const int* __restrict__ pu_ptr, const int* __restrict__ pu_cg,
                                                            const TY* __restrict__ Y, const double* __restrict__ v,
                                                            double* __restrict__ Q) {
    __shared__ double vs[kFoldPairMaxU][64];
    const int g = blockIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), c = threadIdx.x & 63;
    const int i1 = pr_ptr[g + 1];
    int base = pr_ptr[g] + kFoldRows * wave;
    // the coarse rows of the union: wavefront w takes rows 4w .. 4w + 3 (at most 64 in all; one
    // scalar load of their indices from u0 + min(4w, max(nu - 1, 0)), inside the table, which
    // carries 4 padding entries at its end); their loads go out first, then the first pass's
    static_assert(kFoldPairMaxU <= 64, "four union rows per wavefront");
    const int u0 = pu_ptr[g], nu = pu_ptr[g + 1] - u0;
    const int4 cg = *reinterpret_cast<const int4*>(pu_cg + u0 + min(4 * wave, max(nu - 1, 0)));
    const int cgs[4] = {cg.x, cg.y, cg.z, cg.w};
    double vr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        vr[q] = 0.0;
        if (4 * wave + q < nu && c < k) vr[q] = v[(long long)cgs[q] * k + c];
    }
    int4 rec[kFoldRows];
    double side[kFoldRows], fv[kFoldRows];
    int fp[kFoldRows];
    fold_rows_load(base, i1, k, W, c, pr_rec, pr_fpos, pr_fval, Y, rec, side, fp, fv);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (4 * wave + q < nu) vs[4 * wave + q][c] = vr[q];
    __syncthreads();
    fold_rows_store(base, i1, k, c, vs, rec, side, fp, fv, Q);
    for (base += 16 * kFoldRows; base < i1; base += 16 * kFoldRows) {
        fold_rows_load(base, i1, k, W, c, pr_rec, pr_fpos, pr_fval, Y, rec, side, fp, fv);
        fold_rows_store(base, i1, k, c, vs, rec, side, fp, fv, Q);
    }
}

void launch_scatter_fold(const DevTopo& t, int k, int ytype_f32, const void* Y, const double* v, double* Q,
                         hipStream_t st) {
    const long long n = (long long)t.n_lambda * k;
    if (n == 0) return;
    if (k >= 32 && t.n_pairs > 0) {
        if (ytype_f32)
            k_scatter_fold_pair<float><<<t.n_pairs, 1024, 0, st>>>(k, t.fr_w, t.pr_ptr, t.pr_rec, t.fr_pos, t.pr_fval,
                                                                   t.pu_ptr, t.pu_cg, (const float*)Y, v, Q);
        else
            k_scatter_fold_pair<double><<<t.n_pairs, 1024, 0, st>>>(k, t.fr_w, t.pr_ptr, t.pr_rec, t.fr_pos, t.pr_fval,
                                                                    t.pu_ptr, t.pu_cg, (const double*)Y, v, Q);
        return;
    }
    const int grid = (int)((n + 255) / 256);
    if (ytype_f32)
        k_scatter_fold<float><<<grid, 256, 0, st>>>(t.n_lambda, k, t.fr_w, t.row_yo, t.row_sg, (const float*)Y, t.fr_n,
                                                    t.fr_col, t.fr_val, v, Q);
    else
        k_scatter_fold<double><<<grid, 256, 0, st>>>(t.n_lambda, k, t.fr_w, t.row_yo, t.row_sg, (const double*)Y,
                                                     t.fr_n, t.fr_col, t.fr_val, v, Q);
}

// ---------------------------------------------------------------------------------------
// Preconditioner (Sec. 3.1, Eq. 13): x_s = B~^sT r = B^sT W^s r, y_s = S~^s x_s.
// S~^s is symmetric and stored as its upper triangle in 64x64 tiles, so every stored value is
// read once: tile (I, J) adds S_IJ x_J to y_I (row part) and, for I < J, S_IJ^T x_I to y_J
// (column part). Subdomain s is split into G_s parts (work[blockIdx.x] = (s, g, G_s)): part g
// takes tiles [g nt / G_s, (g+1) nt / G_s) in storage order (column block J outer); thread
// (wave, lane) holds row i = 4 wave + lane/16 of a tile and columns 4 (lane%16) .. +3 (one
// 32-byte load per tile, kPsRing tiles ahead). x_s and the partial y_s live in LDS; the column
// part is summed over the tile rows in a fixed order when J changes. With every G_s = 1 the
// parts write y_s; otherwise part g writes ypart + g * nb_tot for k_precond_sum.
constexpr int kPsRing = 8;
typedef double ps4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int tri_col(int t) {   // J with J(J+1)/2 <= t < (J+1)(J+2)/2
    int J = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((J + 1) * (J + 2) / 2 <= t) ++J;
    while (J * (J + 1) / 2 > t) --J;
    return J;
}

// The tiles' storage type TP: double, or float for the FP32 copy of the blocks (the products and
// sums stay FP64: a stored value is converted exactly when it is used).
typedef float ps4f_t __attribute__((ext_vector_type(4)));
template <typename TP>
struct PsRaw;
template <>
struct PsRaw<double> {
    typedef ps4_t raw;
    static __device__ __forceinline__ raw load(__amdgpu_buffer_rsrc_t r, int off) { return load4d(r, off); }
    static __device__ __forceinline__ ps4_t wide(raw a) { return a; }
};
template <>
struct PsRaw<float> {
    typedef ps4f_t raw;
    static __device__ __forceinline__ raw load(__amdgpu_buffer_rsrc_t r, int off) {
        return __builtin_bit_cast(ps4f_t, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    }
    static __device__ __forceinline__ ps4_t wide(raw a) {
        return ps4_t{(double)a[0], (double)a[1], (double)a[2], (double)a[3]};
    }
};

template <typename TP>
__global__ void __launch_bounds__(1024) k_precond_sym(const SubMeta* __restrict__ subs, const int4* __restrict__ work,
                                                      const int* __restrict__ bg_ptr,
                                                      const int* __restrict__ bg_row, const int8_t* __restrict__ bg_sg,
                                                      const double* __restrict__ bg_w, const double* __restrict__ r,
                                                      const TP* __restrict__ Pk, double* __restrict__ y,
                                                      long long ystride, int cap) {
    typedef PsRaw<TP> R;
    constexpr int kTileBytes = 4096 * (int)sizeof(TP);
    extern __shared__ double sh[];
    double* xs = sh;             // cap
    double* ys = sh + cap;       // cap
    double* red = sh + 2 * cap;  // 16 x 64
    const int4 wk = work[blockIdx.x];
    const int s = wk.x, g = wk.y, G = wk.z;
    const SubMeta M = subs[s];
    const int nb = M.n_b, nT = (nb + 63) >> 6, nt = nT * (nT + 1) / 2;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, i = 4 * wave + (lane >> 4), jq = lane & 15;
    // the first tiles' loads go out before the gather of x (they do not depend on it)
    const int t0 = (int)((long long)g * nt / G), t1 = (int)((long long)(g + 1) * nt / G);
    // the part's tiles through a buffer resource: loads past its last tile return zeros, so the
    // ring's loads are unconditional and their waits counted, not drained
    const __amdgpu_buffer_rsrc_t rs =
        rows_rsrc(reinterpret_cast<const double*>(Pk + M.off_Pk + (long long)t0 * 4096), (t1 - t0) * kTileBytes);
    const int toff = (i * 64 + 4 * jq) * (int)sizeof(TP);
    auto ld = [&](int t) -> typename R::raw { return R::load(rs, toff + (t - t0) * kTileBytes); };
    typename R::raw ring[kPsRing];
#pragma unroll
    for (int d = 0; d < kPsRing; ++d) ring[d] = ld(t0 + d);
    for (int q = tid; q < nT * 64; q += 1024) {
        double v = 0.0;
        if (q < nb) {
            const long long gq = M.off_b + q;
            for (int e = bg_ptr[gq]; e < bg_ptr[gq + 1]; ++e) v += bg_sg[e] * bg_w[e] * r[bg_row[e]];
        }
        xs[q] = v;
        ys[q] = 0.0;
    }
    __syncthreads();
    int J = t0 < t1 ? tri_col(t0) : 0, I = t0 - J * (J + 1) / 2;
    double ca[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = t0; t < t1; t += kPsRing) {
#pragma unroll
        for (int d = 0; d < kPsRing; ++d) {
            const ps4_t a = R::wide(ring[d]);
            ring[d] = ld(t + d + kPsRing);
            if (t + d < t1) {   // uniform over the workgroup
                // row part: y_I[i] += sum_b S[i][b] x_J[b]
                const ps4_t xj = *reinterpret_cast<const ps4_t*>(xs + 64 * J + 4 * jq);
                const double rp =
                    row16_sum_dpp(((a[0] * xj[0] + a[1] * xj[1]) + a[2] * xj[2]) + a[3] * xj[3]);   // over jq
                if (jq == 0) ys[64 * I + i] += rp;
                // column part: y_J[b] += S[i][b] x_I[i]
                if (I < J) {
                    const double xi = xs[64 * I + i];
#pragma unroll
                    for (int b = 0; b < 4; ++b) ca[b] = fma(a[b], xi, ca[b]);
                }
                if (I == J || t + d == t1 - 1) {
                    // sum the column part over the 64 tile rows: lanes of equal jq, then wavefronts
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        ca[b] += __shfl_xor(ca[b], 16);
                        ca[b] += __shfl_xor(ca[b], 32);
                    }
                    if (lane < 16)
#pragma unroll
                        for (int b = 0; b < 4; ++b) red[wave * 64 + 4 * lane + b] = ca[b];
                    __syncthreads();
                    if (tid < 64) {
                        double v = 0.0;
#pragma unroll
                        for (int w = 0; w < 16; ++w) v += red[w * 64 + tid];
                        ys[64 * J + tid] += v;
                    }
                    __syncthreads();
#pragma unroll
                    for (int b = 0; b < 4; ++b) ca[b] = 0.0;
                }
                if (++I > J) {
                    ++J;
                    I = 0;
                }
            }
        }
    }
    __syncthreads();
    double* yo = y + (long long)g * ystride + M.off_b;
    for (int q = tid; q < nb; q += 1024) yo[q] = ys[q];
}

// y[q] = sum over g < G_s of ypart[g * n + q], in order (s: the subdomain of b DOF q)
__global__ void k_precond_sum(long long n, const int* __restrict__ bq_s, const int* __restrict__ ps_G,
                              const double* __restrict__ ypart, double* __restrict__ y) {
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int G = ps_G[bq_s[q]];
    double v = 0.0;
    for (int g = 0; g < G; ++g) v += ypart[g * n + q];
    y[q] = v;
}

template <typename TP>
static void precond_local(const DevTopo& t, const double* r, const double* bg_w, const TP* Pk, double* ypart,
                          double* y, hipStream_t st) {
    if (t.nb_tot == 0 || t.ps_nwg == 0) return;
    const int cap = (t.max_nb + 63) / 64 * 64;
    const size_t sh = sizeof(double) * (2 * (size_t)cap + 16 * 64);
    if (t.ps_maxG == 1) {
        k_precond_sym<TP>
            <<<t.ps_nwg, 1024, sh, st>>>(t.subs, t.ps_work, t.bg_ptr, t.bg_row, t.bg_sg, bg_w, r, Pk, y, 0, cap);
    } else {
        k_precond_sym<TP><<<t.ps_nwg, 1024, sh, st>>>(t.subs, t.ps_work, t.bg_ptr, t.bg_row, t.bg_sg, bg_w, r, Pk,
                                                      ypart, t.nb_tot, cap);
        k_precond_sum<<<(int)((t.nb_tot + 255) / 256), 256, 0, st>>>(t.nb_tot, t.bq_s, t.ps_G, ypart, y);
    }
}

void launch_precond_local(const DevTopo& t, const double* r, const double* bg_w, const double* Pk, double* ypart,
                          double* y, hipStream_t st) {
    precond_local(t, r, bg_w, Pk, ypart, y, st);
}

void launch_precond_local32(const DevTopo& t, const double* r, const double* bg_w, const float* Pk32,
                            double* ypart, double* y, hipStream_t st) {
    precond_local(t, r, bg_w, Pk32, ypart, y, st);
}

__global__ void k_round_f32(long long n, const double* __restrict__ a, float* __restrict__ b) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

void launch_round_f32(long long n, const double* a, float* b, hipStream_t st) {
    if (n > 0) k_round_f32<<<(int)((n + 255) / 256), 256, 0, st>>>(n, a, b);
}

// Z[row][c] = sum over the row's sides with g(s) == c of sign * w * y_s[j]  (kz = n_groups or 1).
__global__ void k_precond_scatter(int n_lambda, int kz, int one_column, const int* __restrict__ row_s,
                                  const int* __restrict__ row_j, const int8_t* __restrict__ row_sg,
                                  const SubMeta* __restrict__ subs, const double* __restrict__ w,
                                  const double* __restrict__ y, double* __restrict__ Z) {
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx >= (long long)n_lambda * kz) return;
    // row = idx / kz without a 64-bit division (kz = 64: one wavefront per row)
    const int row = kz == 64 ? (int)(idx >> 6) : kz == 1 ? (int)idx : (int)((unsigned long long)idx / (unsigned)kz);
    const int c = (int)(idx - (long long)row * kz);
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

// kz = 64: a wavefront takes 64 rows; lane l first resolves row r0 + l (its one or two sides:
// group and sign * w * y_s[j]), then the wavefront writes the 64 rows one after another, lane =
// column (coalesced 512-byte rows), taking each row's values by readlane (the row index is
// wavefront-uniform: scalar reads, no LDS round trip). Same sums, same order.
__global__ void __launch_bounds__(256) k_precond_scatter64(int n_lambda, const int* __restrict__ row_s,
                                                           const int* __restrict__ row_j,
                                                           const int8_t* __restrict__ row_sg,
                                                           const SubMeta* __restrict__ subs, const double* __restrict__ w,
                                                           const double* __restrict__ y, double* __restrict__ Z) {
    const int lane = threadIdx.x & 63;
    const int r0 = ((blockIdx.x * 256 + threadIdx.x) >> 6) * 64;
    const int row = r0 + lane;
    int ga = -1, gb = -1;
    double va = 0.0, vb = 0.0;
    if (row < n_lambda) {
        const int s0 = row_s[2 * row], s1 = row_s[2 * row + 1];
        if (s0 >= 0) {
            ga = subs[s0].grp;
            va = row_sg[2 * row] * w[2 * row] * y[subs[s0].off_b + row_j[2 * row]];
        }
        if (s1 >= 0) {
            gb = subs[s1].grp;
            vb = row_sg[2 * row + 1] * w[2 * row + 1] * y[subs[s1].off_b + row_j[2 * row + 1]];
        }
    }
    const int nr = min(64, n_lambda - r0);
    for (int i = 0; i < nr; ++i) {
        const int gai = __builtin_amdgcn_readlane(ga, i), gbi = __builtin_amdgcn_readlane(gb, i);
        const double vai = bcast_lane(va, i), vbi = bcast_lane(vb, i);
        double v = 0.0;
        if (lane == gai) v += vai;
        if (lane == gbi) v += vbi;
        Z[(long long)(r0 + i) * 64 + lane] = v;
    }
}

// Super-lumped preconditioner (Sec. 3.1: S~^s = diag K_bb): y_q = (K_bb)_qq x_q with
// x_q = sum over the multiplier rows of interface DOF q of sign * weight * r_row; one thread per
// interface DOF, the diagonal read from the packed block (diagonal tiles, entry a * 65).
__global__ void __launch_bounds__(256) k_precond_diag(long long nb_tot, const int* __restrict__ bq_s,
                                                      const SubMeta* __restrict__ subs, const int* __restrict__ bg_ptr,
                                                      const int* __restrict__ bg_row, const int8_t* __restrict__ bg_sg,
                                                      const double* __restrict__ bg_w, const double* __restrict__ r,
                                                      const double* __restrict__ Pk, double* __restrict__ y) {
    const long long gq = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (gq >= nb_tot) return;
    const SubMeta& M = subs[bq_s[gq]];
    const int q = (int)(gq - M.off_b), J = q >> 6, a = q & 63;
    const double d = Pk[M.off_Pk + ((long long)J * (J + 1) / 2 + J) * 4096 + a * 65];
    double v = 0.0;
    for (int e = bg_ptr[gq]; e < bg_ptr[gq + 1]; ++e) v += bg_sg[e] * bg_w[e] * r[bg_row[e]];
    y[gq] = d * v;
}

void launch_precond_diag(const DevTopo& t, const double* r, const double* bg_w, const double* Pk, double* y,
                         hipStream_t st) {
    if (t.nb_tot == 0) return;
    k_precond_diag<<<(int)((t.nb_tot + 255) / 256), 256, 0, st>>>(t.nb_tot, t.bq_s, t.subs, t.bg_ptr, t.bg_row,
                                                                    t.bg_sg, bg_w, r, Pk, y);
}

// Keeps only the diagonal of every packed preconditioner block (super-lumped: diag K_bb); one
// workgroup per subdomain over its packed tiles.
__global__ void __launch_bounds__(256) k_pk_diag_only(const SubMeta* __restrict__ subs, double* __restrict__ Pk) {
    const SubMeta& M = subs[blockIdx.x];
    const int nT = (M.n_b + 63) >> 6;
    const long long ne = (long long)nT * (nT + 1) / 2 * 4096;
    for (long long e = threadIdx.x; e < ne; e += blockDim.x) {
        const int tile = (int)(e >> 12), w = (int)(e & 4095);
        int J = 0;
        while ((J + 1) * (J + 2) / 2 <= tile) ++J;
        const int I = tile - J * (J + 1) / 2;
        if (I != J || (w >> 6) != (w & 63)) Pk[M.off_Pk + e] = 0.0;
    }
}

void launch_pk_diag_only(const DevTopo& t, double* Pk, hipStream_t st) {
    if (t.n_sub) k_pk_diag_only<<<t.n_sub, 256, 0, st>>>(t.subs, Pk);
}

void launch_precond_scatter(const DevTopo& t, int one_column, const double* w, const double* y, double* Z,
                            hipStream_t st) {
    const int kz = one_column ? 1 : t.n_groups;
    const long long n = (long long)t.n_lambda * kz;
    if (n == 0) return;
    if (kz == 64) {
        const int nw = (t.n_lambda + 63) / 64;   // wavefronts
        k_precond_scatter64<<<(nw + 3) / 4, 256, 0, st>>>(t.n_lambda, t.row_s, t.row_j, t.row_sg, t.subs, w, y, Z);
        return;
    }
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
    const int row = k == 64 ? (int)(idx >> 6) : (int)((unsigned long long)idx / (unsigned)k), c = (int)(idx - (long long)row * k);
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
