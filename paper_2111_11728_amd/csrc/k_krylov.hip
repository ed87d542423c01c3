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

// ---------------------------------------------------------------------------------------
// Register-direct FP64 matrix-core forms for blocks of 64 directions (the common case).
// Both use the freedom to permute the contraction and output indices consistently so that
// every lane reads 16 or 32 contiguous bytes of a row-major n x 64 operand straight from
// HBM, with a ring of loads in flight; no LDS round trip for the streamed operands.

constexpr int kTsWaves = 8;   // 128 output rows per workgroup

typedef float v4f_t __attribute__((ext_vector_type(4)));

// The 16x16x4 matrix-core step in the two arithmetic types the orthogonalisation runs in. The
// FP32 form reads the same FP64 operands and rounds them in registers; its accumulator rows are
// 4*(lane/16) + v where the FP64 form's are lane/16 + 4v (column lane%16 in both).
template <bool F32> struct MfmaT;
template <> struct MfmaT<false> {
    typedef double T;
    typedef v4d_t V;
    static __device__ __forceinline__ V step(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};
template <> struct MfmaT<true> {
    typedef float T;
    typedef v4f_t V;
    static __device__ __forceinline__ V step(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};


// out = beta C + alpha sum_b A_b Psi_b (A_b = Aptrs[b], n x 64; Psi_b = Mats + 4096 b).
// Wavefront: 16 output rows x 64 columns. Step t = 4 b + q contracts columns 16q..16q+15 of
// A_b: lane (m = lane%16, g = lane/16) supplies A_b[row m][16q + 4g + s] at sub-step s, i.e.
// one 32-byte load per step, issued a whole block (four steps) ahead; Psi_b is staged in LDS
// in the matching operand order (FP32: ((q*4 + j)*64 + lane)*4 + s; FP64: (((q*4 + j)*2 + s/2)*64
// + lane)*2 + s%2, so that each 16-byte read has a 16-byte lane stride) <- Psi_b[16q + 4g + s][16j + m],
// double-buffered per block. F32: products on the FP32 matrix cores (Psi_b staged rounded to
// FP32, A_b rounded as it is loaded), sums in FP32 per row, the update C + alpha acc in FP64.
// (at most 128 VGPRs: four wavefronts per SIMD, two workgroups per CU)
template <bool F32>
__global__ void __launch_bounds__(64 * kTsWaves) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_ts64(int n, int nblk, const double* const* __restrict__ Aptrs,
                                                        const double* __restrict__ Mats, const double* C, double* out,
                                                        double alpha, double beta, const double* const* Aptrs2,
                                                        double* out2, const int* __restrict__ rb_design,
                                                        long long mstride) {
    if (blockIdx.y) {   // second job of a paired launch: same Mats, its own operands
        Aptrs = Aptrs2;
        out = out2;
    }
    // several designs: the matrices of the design owning this workgroup's rows (a 256-row block)
    if (rb_design) Mats += (long long)rb_design[(blockIdx.x * (16 * kTsWaves)) >> 8] * mstride;
    typedef typename MfmaT<F32>::T T;
    typedef typename MfmaT<F32>::V V;
    __shared__ __attribute__((aligned(16))) T Ps[2][4096];
    const int tid = threadIdx.x, lane = tid & 63, m = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rb0 = blockIdx.x * (16 * kTsWaves) + 16 * wave;
    const int nbytes = max(0, min(16, n - rb0)) * 512;   // this wavefront's rows of every A_b
    const int aoff = m * 512 + 32 * g;                     // + 128 q for column block q
    constexpr int kPer = 4096 / (64 * kTsWaves);
    T pst[kPer];
    auto load_psi = [&](int b) {
        const double* P = Mats + (long long)b * 4096;
#pragma unroll
        for (int u = 0; u < kPer; ++u) pst[u] = (T)P[tid + 64 * kTsWaves * u];
    };
    auto store_psi = [&](T* Pb) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 64 * kTsWaves * u, kr = e >> 6, kc = e & 63;
            const int qj = (kr >> 4) * 4 + (kc >> 4), ln = ((kr & 15) >> 2) * 16 + (kc & 15), sub = kr & 3;
            if constexpr (F32)   // one 16-byte operand group per lane
                Pb[(qj * 64 + ln) * 4 + sub] = pst[u];
            else   // sub-steps {0,1} and {2,3} in separate planes: 16-byte lane stride, no bank conflicts
                Pb[((qj * 2 + (sub >> 1)) * 64 + ln) * 2 + (sub & 1)] = pst[u];
        }
    };
    // block b's rows of this wavefront (no bytes past the last block)
    auto rsrc_of = [&](int b) {
        return rows_rsrc(Aptrs[min(b, nblk - 1)] + (long long)rb0 * 64, b < nblk ? nbytes : 0);
    };
    V acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = V{0, 0, 0, 0};
    v4d_t ring[4];
    __amdgpu_buffer_rsrc_t ra = rsrc_of(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) ring[q] = load4d(ra, aoff + 128 * q);
    load_psi(0);
    store_psi(Ps[0]);
    __syncthreads();
    for (int b = 0; b < nblk; ++b) {
        if (b + 1 < nblk) load_psi(b + 1);
        const T* Pb = Ps[b & 1];
        ra = rsrc_of(b + 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const v4d_t a = ring[q];
            ring[q] = load4d(ra, aoff + 128 * q);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                V bv;
                if constexpr (F32) {
                    bv = *reinterpret_cast<const V*>(Pb + ((q * 4 + j) * 64 + lane) * 4);
                } else {
                    const v2d_t b0 = *reinterpret_cast<const v2d_t*>(Pb + (((q * 4 + j) * 2) * 64 + lane) * 2);
                    const v2d_t b1 = *reinterpret_cast<const v2d_t*>(Pb + (((q * 4 + j) * 2 + 1) * 64 + lane) * 2);
                    bv = V{b0[0], b0[1], b1[0], b1[1]};
                }
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) acc[j] = MfmaT<F32>::step(a[s2], bv[s2], acc[j]);
            }
        }
        if (b + 1 < nblk) store_psi(Ps[(b + 1) & 1]);
        __syncthreads();
    }
    // D layout: lane holds rows MfmaT::row(g, v), column m of each 16x16 block j
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = rb0 + MfmaT<F32>::row(g, v);
        if (row >= n) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long idx = (long long)row * 64 + 16 * j + m;
            out[idx] = (beta == 0.0 ? 0.0 : beta * C[idx]) + alpha * (double)acc[j][v];
        }
    }
}

constexpr int kGrRing = 6;    // 4-row steps in flight per lane
constexpr int kGrGroups = 256; // workgroups per round: one per CU

// Gram products Psi_b = A_b^T B for 64 directions over all blocks b < nblk at once. Blocks
// are taken in pairs (b = 2p, 2p+1) that share every load of B: the npair * nsteps 4-row steps
// (pair-major) are split evenly over the G workgroups (G a multiple of 256, so no range spans
// more than two pairs); within a workgroup the four wavefronts split each pair segment and
// every wavefront accumulates two full 64 x 64 results (32 FP64 16x16 accumulators, one
// wavefront per SIMD, loads kGrRing steps ahead; F32: FP32 matrix cores on the operands rounded
// in registers, FP32 sums over the wavefront's rows). Rows/columns are permuted so that at step
// st lane (m, g) loads A_b[4 st + g][4m..4m+3] and B[4 st + g][4m..4m+3]: accumulator row m'
// of block ib is A column 4 m' + ib, column n' of block jb is B column 4 n' + jb. The
// wavefront results meet in LDS (fixed order); segment slot t of workgroup w writes, for its
// pair p, part[((w*2 + t)*2 + h)*4096 + i*64 + j] for block 2p + h.
// Several designs (segs != null): design d owns max(npair, segs[d].base) consecutive
// workgroups, which split its own rows in the same way; partials keep the global workgroup index.
// The design of workgroup wg: w[d] <= wg < w[d + 1] (w: first workgroup of each design, built on
// the host per launch and passed by value)
__device__ __forceinline__ int seg_of(const SegBases& sb, int nseg, int wg) {
    int d = 0;
    while (d + 1 < nseg && sb.w[d + 1] <= wg) ++d;
    return d;
}

template <bool F32>
__global__ void __launch_bounds__(256, 1) k_gram64(int n, int nblk, const double* const* __restrict__ Aptrs,
                                                   const double* __restrict__ B, double* __restrict__ part,
                                                   const KrySeg* __restrict__ segs, int nseg, SegBases sb) {
    __shared__ double red[4 * 4096];
    const int wg = blockIdx.x;
    int G = gridDim.x, w = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, m = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int npair = (nblk + 1) >> 1;
    long long arow0 = 0;   // first element of this workgroup's design in every n x 64 block
    if (segs) {
        const int d = seg_of(sb, nseg, wg);
        w = wg - sb.w[d];
        G = sb.w[d + 1] - sb.w[d];
        arow0 = (long long)segs[d].row0 * 64;
        n = segs[d].nrows;
        B += arow0;
    }
    const long long nsteps = (n + 3) >> 2, S = nsteps * npair;
    const long long s_lo = (long long)w * S / G, s_hi = (long long)(w + 1) * S / G;
    for (int slot = 0; slot < 2; ++slot) {
        const long long p_ll = s_lo / nsteps + slot;
        if (p_ll >= npair || p_ll * nsteps >= s_hi) break;
        const int pr = (int)p_ll;
        const long long a0 = std::max(s_lo, p_ll * nsteps) - p_ll * nsteps;
        const long long a1 = std::min(s_hi, (p_ll + 1) * nsteps) - p_ll * nsteps;
        const int w0 = (int)(a0 + (a1 - a0) * wave / 4), w1 = (int)(a0 + (a1 - a0) * (wave + 1) / 4);
        const double* A0 = Aptrs[2 * pr] + arow0;
        const bool has1 = 2 * pr + 1 < nblk;
        const double* A1 = has1 ? Aptrs[2 * pr + 1] + arow0 : A0;
        typedef typename MfmaT<F32>::V V;
        V acc[2][4][4];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[h][i][j] = V{0, 0, 0, 0};
        v4d_t ar0[kGrRing], ar1[kGrRing], br[kGrRing];
        // rows [4 w0, min(4 w1, n)) of the three operands
        const long long row_lo = 4LL * w0;
        const int nbytes = (int)std::max(0LL, std::min((long long)n, 4LL * w1) - row_lo) * 512;
        const __amdgpu_buffer_rsrc_t rA0 = rows_rsrc(A0 + row_lo * 64, nbytes);
        const __amdgpu_buffer_rsrc_t rA1 = rows_rsrc(A1 + row_lo * 64, has1 ? nbytes : 0);
        const __amdgpu_buffer_rsrc_t rB = rows_rsrc(B + row_lo * 64, nbytes);
        auto ld = [&](int st, v4d_t& av0, v4d_t& av1, v4d_t& bv) {
            const int off = ((st - w0) * 4 + g) * 512 + 32 * m;
            av0 = load4d(rA0, off);
            av1 = load4d(rA1, off);
            bv = load4d(rB, off);
        };
#pragma unroll
        for (int d = 0; d < kGrRing; ++d) ld(w0 + d, ar0[d], ar1[d], br[d]);
        auto prod2 = [&](int d) {
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) {
                    acc[0][ib][jb] = MfmaT<F32>::step(ar0[d][ib], br[d][jb], acc[0][ib][jb]);
                    acc[1][ib][jb] = MfmaT<F32>::step(ar1[d][ib], br[d][jb], acc[1][ib][jb]);
                }
        };
        auto prod1 = [&](int d) {   // a single block (the last one of an odd count)
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
                    acc[0][ib][jb] = MfmaT<F32>::step(ar0[d][ib], br[d][jb], acc[0][ib][jb]);
        };
        // whole rings without guards: steps past the range load zeros and add nothing, so the
        // last ring runs in full (at most kGrRing - 1 idle steps per wavefront)
        if (has1) {
            for (int st = w0; st < w1; st += kGrRing) {
#pragma unroll
                for (int d = 0; d < kGrRing; ++d) {
                    prod2(d);
                    ld(st + d + kGrRing, ar0[d], ar1[d], br[d]);
                }
            }
        } else {
            for (int st = w0; st < w1; st += kGrRing) {
#pragma unroll
                for (int d = 0; d < kGrRing; ++d) {
                    prod1(d);
                    ld(st + d + kGrRing, ar0[d], ar1[d], br[d]);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && !has1) break;
            // D layout: lane holds rows MfmaT::row(g, v), column m of block (ib, jb)
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        red[wave * 4096 + (4 * MfmaT<F32>::row(g, v) + ib) * 64 + 4 * m + jb] =
                            (double)acc[h][ib][jb][v];
            __syncthreads();
            double* out = part + (((long long)wg * 2 + slot) * 2 + h) * 4096;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = tid + 256 * u;
                out[e] = ((red[e] + red[4096 + e]) + red[8192 + e]) + red[12288 + e];
            }
            __syncthreads();
        }
    }
}

// out[b][e] = sum of the segment partials of block b (pair b/2, half b%2): workgroup = 64
// consecutive entries of one block; its W wavefronts take every W-th contributing workgroup
// (loads independent, in flight together) and meet in LDS in a fixed order. W = 16 when a
// block has many contributors (few stored blocks), 4 otherwise.
template <int W>
__global__ void __launch_bounds__(64 * W) k_gram64_reduce(int n, int nblk, int G, const double* __restrict__ part,
                                                          double* __restrict__ out, const KrySeg* __restrict__ segs,
                                                          int nseg, SegBases sb) {
    __shared__ double red[W][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int bid = blockIdx.x, wbase = 0;
    const int npair = (nblk + 1) >> 1;
    if (segs) {   // workgroup = (design, block, 64 entries); that design's workgroups only
        const int d = bid / (nblk * 64);
        bid -= d * nblk * 64;
        wbase = sb.w[d];
        G = sb.w[d + 1] - sb.w[d];
        n = segs[d].nrows;
        out += (long long)d * nblk * 4096;
    }
    const int b = bid >> 6, e = ((bid & 63) << 6) + lane;
    const int pr = b >> 1, h = b & 1;
    const long long nsteps = (n + 3) >> 2, S = nsteps * npair;
    const long long bs = (long long)pr * nsteps, be = bs + nsteps;
    // contributing workgroups wf..wl: [w S / G, (w+1) S / G) meets [bs, be); only wf can
    // start before bs (its pair-pr partial is then in slot 1)
    long long wf = bs * G / S;
    while (wf > 0 && wf * S / G > bs) --wf;
    while ((wf + 1) * S / G <= bs) ++wf;
    long long wl = (be * G + S - 1) / S;
    if (wl > G - 1) wl = G - 1;
    while (wl > wf && wl * S / G >= be) --wl;
    const int slot_f = wf * S / G < bs ? 1 : 0;
    // with at least as many steps as workgroups every range is non-empty; otherwise a
    // workgroup with an empty range wrote nothing and adds nothing
    const bool dense = S >= G;
    double v = 0.0;
#pragma unroll 4
    for (long long ww = wf + wave; ww <= wl; ww += W)
        if (dense || (ww + 1) * S / G > ww * S / G)
            v += part[(((wbase + ww) * 2 + (ww == wf ? slot_f : 0)) * 2 + h) * 4096 + e];
    red[wave][lane] = v;
    __syncthreads();
    if (wave == 0) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < W; ++q) t += red[q][lane];
        out[(long long)b * 4096 + e] = t;
    }
}

// contrib: about how many workgroup partials each entry sums
static void launch_gram64_reduce(int nwg, int contrib, int n, int nblk, int G, const double* part, double* out,
                                 const KrySeg* segs, int nseg, const SegBases& sb, hipStream_t st) {
    if (contrib >= 32)
        k_gram64_reduce<16><<<nwg, 64 * 16, 0, st>>>(n, nblk, G, part, out, segs, nseg, sb);
    else
        k_gram64_reduce<4><<<nwg, 64 * 4, 0, st>>>(n, nblk, G, part, out, segs, nseg, sb);
}

// part[c][0..63] = sum over the chunk's rows of A[row][:] * x[row] (A: n x 64). Lane = column;
// a wavefront covers 8 rows per pass (the loads of two passes in flight), four wavefronts summed
// in LDS (fixed order).
__global__ void __launch_bounds__(256) k_gemv_t64(int n, const double* __restrict__ A, const double* __restrict__ x,
                                                  double* __restrict__ part) {
    __shared__ double red[4][64];
    const int c = blockIdx.x, nchunk = gridDim.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r0 = (int)((long long)c * n / nchunk), r1 = (int)((long long)(c + 1) * n / nchunk);
    double acc = 0.0;
    for (int rr = r0 + 8 * wave; rr < r1; rr += 64) {
        double av[16], xv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int row = rr + (u < 8 ? u : 24 + u);   // this pass's 8 rows, then the next pass's
            av[u] = row < r1 ? A[(long long)row * 64 + lane] : 0.0;
            xv[u] = row < r1 ? x[row] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) acc = fma(av[u], xv[u], acc);
    }
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) part[(long long)c * 64 + lane] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// lam += W g; r -= Q g for 64 directions: 16 lanes per row, 4 consecutive columns each.
// lam_out = lam + W gamma and r -= Q gamma (lam_out may be lam itself)
__global__ void __launch_bounds__(256) k_update_lr64(int n, const double* __restrict__ W, const double* __restrict__ Q,
                                                     const double* __restrict__ gm, const double* lam,
                                                     double* lam_out, double* __restrict__ r,
                                                     const int* __restrict__ rb_design) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int row = (int)(t >> 4), p = (int)(t & 15);
    // several designs: the gamma of the row's design
    if (rb_design && row < n) gm += rb_design[row >> 8] * 64;
    const v4d_t gv = *reinterpret_cast<const v4d_t*>(gm + 4 * p);
    double dl = 0.0, dr = 0.0;
    if (row < n) {
        const v4d_t w = *reinterpret_cast<const v4d_t*>(W + (long long)row * 64 + 4 * p);
        dl = ((w[0] * gv[0] + w[1] * gv[1]) + w[2] * gv[2]) + w[3] * gv[3];
        if (Q) {
            const v4d_t q = *reinterpret_cast<const v4d_t*>(Q + (long long)row * 64 + 4 * p);
            dr = ((q[0] * gv[0] + q[1] * gv[1]) + q[2] * gv[2]) + q[3] * gv[3];
        }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        dl += __shfl_xor(dl, o, 16);
        dr += __shfl_xor(dr, o, 16);
    }
    if (row < n && p == 0) {
        lam_out[row] = lam[row] + dl;
        if (Q) r[row] -= dr;
    }
}

// part[block] = sum over rows of r[row] * sum_c Z[row][c] for 64 columns: 16 lanes per row.
__global__ void __launch_bounds__(256) k_rowsum_dot64(int n, const double* __restrict__ r, const double* __restrict__ Z,
                                                      double* __restrict__ part) {
    __shared__ double red[4];
    double acc = 0.0;
    for (long long t = blockIdx.x * 256LL + threadIdx.x; t < 16LL * n; t += 256LL * gridDim.x) {
        const int row = (int)(t >> 4), p = (int)(t & 15);
        const v4d_t z = *reinterpret_cast<const v4d_t*>(Z + (long long)row * 64 + 4 * p);
        acc = fma(r[row], ((z[0] + z[1]) + z[2]) + z[3], acc);
    }
    acc = warp_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

void launch_ts_gemm(int n, int kd, int nblk, const double* const* Aptrs, const double* Mats, const double* C,
                    double* out, double alpha, double beta, hipStream_t st, bool f32) {
    if (!n || !nblk) return;
    const int nwg = (n + 16 * kTsWaves - 1) / (16 * kTsWaves);
    if (kd == 64 && f32)
        k_ts64<true><<<nwg, 64 * kTsWaves, 0, st>>>(n, nblk, Aptrs, Mats, C, out, alpha, beta, nullptr, nullptr, nullptr,
                                                    0);
    else if (kd == 64)
        k_ts64<false><<<nwg, 64 * kTsWaves, 0, st>>>(n, nblk, Aptrs, Mats, C, out, alpha, beta, nullptr, nullptr,
                                                     nullptr, 0);
    else
        k_ts_gemm<<<(n + 63) / 64, 256, 0, st>>>(n, kd, nblk, Aptrs, Mats, C, out, alpha, beta);
}

void launch_ts_pair(int n, int kd, const double* const* Aptrs, const double* const* Aptrs2, const double* Mats,
                    double* out, double* out2, hipStream_t st) {
    if (!n) return;
    if (kd == 64) {
        k_ts64<false><<<dim3((n + 16 * kTsWaves - 1) / (16 * kTsWaves), 2), 64 * kTsWaves, 0, st>>>(
            n, 1, Aptrs, Mats, nullptr, out, 1.0, 0.0, Aptrs2, out2, nullptr, 0);
        return;
    }
    launch_ts_gemm(n, kd, 1, Aptrs, Mats, nullptr, out, 1.0, 0.0, st);
    launch_ts_gemm(n, kd, 1, Aptrs2, Mats, nullptr, out2, 1.0, 0.0, st);
}

void launch_gram(int n, int ka, int kb, const double* const* Aptrs, int nblk, const double* B, double* part,
                 double* out, hipStream_t st, bool f32) {
    if (nblk == 0) return;
    if (ka == 64 && kb == 64 && n >= 64) {
        const int npair = (nblk + 1) / 2;
        const int G = kGrGroups * ((npair + kGrGroups - 1) / kGrGroups);
        if ((long long)G * 4 * 4096 > kGramPartCap) throw std::length_error("Gram partial buffer too small");
        const SegBases none{};
        if (f32)
            k_gram64<true><<<G, 256, 0, st>>>(n, nblk, Aptrs, B, part, nullptr, 0, none);
        else
            k_gram64<false><<<G, 256, 0, st>>>(n, nblk, Aptrs, B, part, nullptr, 0, none);
        launch_gram64_reduce(nblk * 64, G / npair, n, nblk, G, part, out, nullptr, 0, none, st);
        return;
    }
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
// a[p] for a wavefront-uniform p: a scalar branch to one register move (no LDS round trip)
__device__ __forceinline__ double pick64(const double (&a)[64], int p) {
    switch (p) {
        case 0: return a[0];
        case 1: return a[1];
        case 2: return a[2];
        case 3: return a[3];
        case 4: return a[4];
        case 5: return a[5];
        case 6: return a[6];
        case 7: return a[7];
        case 8: return a[8];
        case 9: return a[9];
        case 10: return a[10];
        case 11: return a[11];
        case 12: return a[12];
        case 13: return a[13];
        case 14: return a[14];
        case 15: return a[15];
        case 16: return a[16];
        case 17: return a[17];
        case 18: return a[18];
        case 19: return a[19];
        case 20: return a[20];
        case 21: return a[21];
        case 22: return a[22];
        case 23: return a[23];
        case 24: return a[24];
        case 25: return a[25];
        case 26: return a[26];
        case 27: return a[27];
        case 28: return a[28];
        case 29: return a[29];
        case 30: return a[30];
        case 31: return a[31];
        case 32: return a[32];
        case 33: return a[33];
        case 34: return a[34];
        case 35: return a[35];
        case 36: return a[36];
        case 37: return a[37];
        case 38: return a[38];
        case 39: return a[39];
        case 40: return a[40];
        case 41: return a[41];
        case 42: return a[42];
        case 43: return a[43];
        case 44: return a[44];
        case 45: return a[45];
        case 46: return a[46];
        case 47: return a[47];
        case 48: return a[48];
        case 49: return a[49];
        case 50: return a[50];
        case 51: return a[51];
        case 52: return a[52];
        case 53: return a[53];
        case 54: return a[54];
        case 55: return a[55];
        case 56: return a[56];
        case 57: return a[57];
        case 58: return a[58];
        case 59: return a[59];
        case 60: return a[60];
        case 61: return a[61];
        case 62: return a[62];
        case 63: return a[63];
        default: return 0.0;
    }
}

// max over the wavefront of a double: DPP within rows of 16 (xor 1, xor 2, rotate 4, rotate 8;
// dpp_mov), then the four row maxima through readlane (uniform result)
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_mov<0xB1>(v));    // quad_perm [1,0,3,2]
    v = fmax(v, dpp_mov<0x4E>(v));    // quad_perm [2,3,0,1]
    v = fmax(v, dpp_mov<0x124>(v));   // row_ror:4
    v = fmax(v, dpp_mov<0x128>(v));   // row_ror:8
    auto rl = [&](int lane) {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    };
    return fmax(fmax(rl(0), rl(16)), fmax(rl(32), rl(48)));
}

// a[p] = v for a wavefront-uniform p (scalar branch to one register move)
#define FETI_PUT1(i) \
    case i:          \
        a[i] = v;    \
        break;
#define FETI_PUT8(i) FETI_PUT1(i) FETI_PUT1(i + 1) FETI_PUT1(i + 2) FETI_PUT1(i + 3) FETI_PUT1(i + 4) FETI_PUT1(i + 5) FETI_PUT1(i + 6) FETI_PUT1(i + 7)
__device__ __forceinline__ void put64(double (&a)[64], int p, double v) {
    switch (p) {
        FETI_PUT8(0) FETI_PUT8(8) FETI_PUT8(16) FETI_PUT8(24) FETI_PUT8(32) FETI_PUT8(40) FETI_PUT8(48) FETI_PUT8(56)
        default: break;
    }
}
#undef FETI_PUT8
#undef FETI_PUT1

// The columns of Ltilde^{-T} are built during the factorisation, in the original index space:
// with pivot p at step m, the direction t_m = N^T (Ltilde^{-T})[:, m] obeys
//     t_m = (e_p - sum_{q<m} L_q[p] t_q) / piv_m,
// L_q the factor column of step q (forward substitution for row m of Ltilde^{-1}), so the pivot
// order is never needed; T[l][q] = s_l t_q[l]. Two wavefronts: wavefront 0 factorises (lane l
// keeps column l of the working matrix in registers), wavefront 1 builds the t_q (lane l keeps
// t_q[l]); they meet once per step at a barrier, both loops running the same number of
// barriers (each leaves after reading the same stop mark p_s[m] < 0).
__global__ void __launch_bounds__(128) k_pivchol(int k, const double* __restrict__ D, double rr_tol,
                                                 double* __restrict__ T, int* __restrict__ rank_out,
                                                 unsigned long long* __restrict__ mask_out) {
    __shared__ __attribute__((aligned(16))) double Lm[64][66];    // Lm[m][i]: entry i of factor column m
    __shared__ __attribute__((aligned(16))) double LmT[64][66];   // LmT[i][m] = Lm[m][i]
    __shared__ double scs[64];
    __shared__ double ipv_s[64];
    __shared__ int p_s[64];
    // one workgroup per design in the segmented form (grid = designs)
    D += (long long)blockIdx.x * k * k;
    T += (long long)blockIdx.x * k * k;
    rank_out += blockIdx.x;
    if (mask_out) mask_out += blockIdx.x;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    // D staged through LDS by coalesced rows; all 32 loads of a lane are in flight together
    // (entries outside the k x k matrix read as zeros from the buffer resource)
    {
        const __amdgpu_buffer_rsrc_t rd = rows_rsrc(D, k * k * 8);
        double v[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int i = 32 * w + u;
            v[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rd, l < k ? (i * k + l) * 8 : k * k * 8, 0, 0));
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) Lm[32 * w + u][l] = v[u];
    }
    __syncthreads();
    if (w == 0) {
        double a[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) a[i] = 0.5 * (Lm[i][l] + Lm[l][i]);
        const double dg = l < k ? 0.5 * (Lm[l][l] + Lm[l][l]) : -1.0;
        const double dmax = wave_max(dg);
        const bool live = l < k && dmax > 0.0 && dg > 1e-30 * dmax;
        const double sc = live ? 1.0 / sqrt(dg) : 0.0;
        scs[l] = sc;
        __syncthreads();   // (S) scs complete, Lm free, LmT zeroed
#pragma unroll
        for (int i = 0; i < 64; ++i) a[i] = a[i] * scs[i] * sc;
        double diag = dg * sc * sc;   // = a[l]
        bool rem = live;
        for (int m = 0; m < k; ++m) {
            // largest remaining pivot, lowest index on ties
            const double cand = rem ? diag : -1.0e300;
            const double best = wave_max(cand);
            const bool go = best > rr_tol;
            const unsigned long long hit = __ballot(cand == best);
            const int p = go ? __builtin_amdgcn_readfirstlane(__ffsll((long long)hit) - 1) : -1;
            double lc = 0.0;
            if (go) {
                const double piv = sqrt(best);
                const double ipiv = 1.0 / piv;
                // A[l][p] = A[p][l] (symmetric among the remaining indices) = a[p] of lane l
                lc = (l == p) ? piv : (rem ? pick64(a, p) * ipiv : 0.0);
                if (l == p) rem = false;
                Lm[m][l] = lc;
                LmT[l][m] = lc;
                if (l == 0) ipv_s[m] = ipiv;
            }
            if (l == 0) p_s[m] = p;
            __syncthreads();   // (B_m)
            if (!go) break;
            // Schur-complement update of the remaining columns: A[i][l] -= lc_i lc_l
            // (the column is read in two batches of sixteen 16-byte loads, all in flight together)
            if (rem) {
#pragma unroll
                for (int h = 0; h < 64; h += 32) {
                    double2 c2[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) c2[u] = *reinterpret_cast<const double2*>(&Lm[m][h + 2 * u]);
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        a[h + 2 * u] -= c2[u].x * lc;
                        a[h + 2 * u + 1] -= c2[u].y * lc;
                    }
                }
                diag -= lc * lc;
            }
        }
    } else {
        double x[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) {
            x[i] = 0.0;
            LmT[l][i] = 0.0;
        }
        __syncthreads();   // (S)
        int m = 0;
        for (; m < k; ++m) {
            __syncthreads();   // (B_m)
            const int p = p_s[m];
            if (p < 0) break;
            // LmT[p][q] = L_q[p] for q < m; entries q > m are zero (later steps write zeros
            // into row p: index p is no longer a candidate) and x[m] is still zero
            // (row p in two batches of sixteen 16-byte loads in flight together, four partial sums)
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
            for (int h = 0; h < 64; h += 32) {
                double2 bq[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) bq[u] = *reinterpret_cast<const double2*>(&LmT[p][h + 2 * u]);
#pragma unroll
                for (int u = 0; u < 16; u += 2) {
                    s0 = fma(bq[u].x, x[h + 2 * u], s0);
                    s1 = fma(bq[u].y, x[h + 2 * u + 1], s1);
                    s2 = fma(bq[u + 1].x, x[h + 2 * u + 2], s2);
                    s3 = fma(bq[u + 1].y, x[h + 2 * u + 3], s3);
                }
            }
            put64(x, m, ((l == p ? 1.0 : 0.0) - ((s0 + s1) + (s2 + s3))) * ipv_s[m]);
        }
        const int rank = m;
        // row l of T; components of indices never taken as pivots are exactly zero
        if (l < k) {
            const double s = scs[l];
#pragma unroll
            for (int j = 0; j < 64; ++j)
                if (j < k) T[l * k + j] = j < rank ? s * x[j] : 0.0;
        }
        if (l == 0) {
            *rank_out = rank;
            if (mask_out) {   // bit j: column j was taken as a pivot (kept)
                unsigned long long msk = 0;
                for (int q = 0; q < rank; ++q) msk |= 1ull << p_s[q];
                *mask_out = msk;
            }
        }
    }
}

// n scalars into host-mapped memory, then the sequence number seq after them, behind a
// system-scope fence: a host that reads seq there also reads the scalars (one wavefront)
__global__ void __launch_bounds__(64) k_publish(const double* __restrict__ src, int n, double* dst, long long seq) {
    for (int i = threadIdx.x; i < n; i += 64) dst[i] = src[i];
    __threadfence_system();
    if (threadIdx.x == 0) *reinterpret_cast<volatile long long*>(dst + n) = seq;
}

void launch_publish(const double* src, int n, double* dst, long long seq, hipStream_t st) {
    k_publish<<<1, 64, 0, st>>>(src, n, dst, seq);
}

void launch_pivchol(int k, const double* D, double rr_tol, double* T, int* rank, hipStream_t st,
                    unsigned long long* kept_mask) {
    k_pivchol<<<1, 128, 0, st>>>(k, D, rr_tol, T, rank, kept_mask);
}

// ---- segmented forms (several designs, each with its own directions in the 64 columns) ----
void launch_gram_seg(const DevTopo& t, int n, const double* const* Aptrs, int nblk, const double* B, double* part,
                     double* out, hipStream_t st, bool f32) {
    if (nblk == 0) return;
    const int nseg = (int)t.hkseg.size();
    const int npair = (nblk + 1) / 2;
    if (nseg > kMaxSegDesigns) throw std::length_error("too many designs for a segmented Gram product");
    SegBases sb{};
    for (int d = 0; d < nseg; ++d) sb.w[d + 1] = sb.w[d] + std::max(npair, t.hkseg[d].base);
    const int G = sb.w[nseg];
    if ((long long)G * 4 * 4096 > kGramPartCap) throw std::length_error("Gram partial buffer too small");
    (void)n;
    if (f32)
        k_gram64<true><<<G, 256, 0, st>>>(0, nblk, Aptrs, B, part, t.kseg, nseg, sb);
    else
        k_gram64<false><<<G, 256, 0, st>>>(0, nblk, Aptrs, B, part, t.kseg, nseg, sb);
    launch_gram64_reduce(nseg * nblk * 64, G / (nseg * npair), 0, nblk, G, part, out, t.kseg, nseg, sb, st);
}

void launch_ts_seg(const DevTopo& t, int n, int nblk, const double* const* Aptrs, const double* Mats, long long mstride,
                   const double* C, double* out, double alpha, double beta, hipStream_t st, bool f32) {
    if (!n || !nblk) return;
    const int nwg = (n + 16 * kTsWaves - 1) / (16 * kTsWaves);
    if (f32)
        k_ts64<true><<<nwg, 64 * kTsWaves, 0, st>>>(n, nblk, Aptrs, Mats, C, out, alpha, beta, nullptr, nullptr,
                                                    t.rb_design, mstride);
    else
        k_ts64<false><<<nwg, 64 * kTsWaves, 0, st>>>(n, nblk, Aptrs, Mats, C, out, alpha, beta, nullptr, nullptr,
                                                     t.rb_design, mstride);
}

void launch_ts_pair_seg(const DevTopo& t, int n, const double* const* Aptrs, const double* const* Aptrs2,
                        const double* Mats, double* out, double* out2, hipStream_t st) {
    if (!n) return;
    k_ts64<false><<<dim3((n + 16 * kTsWaves - 1) / (16 * kTsWaves), 2), 64 * kTsWaves, 0, st>>>(
        n, 1, Aptrs, Mats, nullptr, out, 1.0, 0.0, Aptrs2, out2, t.rb_design, 4096);
}

// out[d*64 + e] = sum of the 256-row chunk partials of design d, in chunk order (16 wavefronts,
// fixed-order combine)
__global__ void __launch_bounds__(1024) k_colsum64_seg(const KrySeg* __restrict__ segs, const double* __restrict__ part,
                                                       double* __restrict__ out) {
    __shared__ double red[16][64];
    const int d = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c0 = segs[d].row0 >> 8, c1 = (segs[d].row0 + segs[d].nrows) >> 8;
    double v = 0.0;
    for (int c = c0 + wave; c < c1; c += 16) v += part[(long long)c * 64 + lane];
    red[wave][lane] = v;
    __syncthreads();
    if (wave == 0) {
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < 16; ++w) tot += red[w][lane];
        out[(long long)d * 64 + lane] = tot;
    }
}

void launch_gemv_t_seg(const DevTopo& t, int n, const double* A, const double* x, double* part, double* out,
                       hipStream_t st) {
    if (!n) return;
    const int nchunk = n / 256;   // 256-row chunks: each lies in one design
    k_gemv_t64<<<nchunk, 256, 0, st>>>(n, A, x, part);
    k_colsum64_seg<<<(int)t.hkseg.size(), 1024, 0, st>>>(t.kseg, part, out);
}

void launch_update_lr_seg(const DevTopo& t, int n, const double* W, const double* Q, const double* g, double* lam,
                          double* r, hipStream_t st) {
    if (n) k_update_lr64<<<(int)((16LL * n + 255) / 256), 256, 0, st>>>(n, W, Q, g, lam, lam, r, t.rb_design);
}

void launch_pivchol_seg(int nseg, const double* D, double rr_tol, double* T, int* rank, unsigned long long* kept_mask,
                        hipStream_t st) {
    k_pivchol<<<nseg, 128, 0, st>>>(64, D, rr_tol, T, rank, kept_mask);
}

// Z[row][:] = 0 for the rows of the designs set in frozen (bit d = design d)
__global__ void k_zero_rows(long long n, const int* __restrict__ rb_design, unsigned long long frozen,
                            double* __restrict__ Z) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= n * 64) return;
    if ((frozen >> rb_design[(e >> 6) >> 8]) & 1ull) Z[e] = 0.0;
}

void launch_zero_rows(const DevTopo& t, int n, unsigned long long frozen, double* Z, hipStream_t st) {
    if (frozen && n) k_zero_rows<<<(int)((64LL * n + 255) / 256), 256, 0, st>>>(n, t.rb_design, frozen, Z);
}

// Z[row][c] = 0 for every column c with bit c of mask set (n x k, k <= 64)
__global__ void k_zero_cols(long long n, int k, unsigned long long mask, double* __restrict__ Z) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int c = (int)(e % k);
    if ((mask >> c) & 1ull) Z[e] = 0.0;
}

void launch_zero_cols(long long n, int k, unsigned long long mask, double* Z, hipStream_t st) {
    if (mask && n) k_zero_cols<<<(int)((n * k + 255) / 256), 256, 0, st>>>(n, k, mask, Z);
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
                            const double* __restrict__ g, const double* lam, double* lam_out, double* __restrict__ r) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    double dl = 0.0, dr = 0.0;
    for (int q = 0; q < k; ++q) {
        dl += W[(long long)row * k + q] * g[q];
        if (Q) dr += Q[(long long)row * k + q] * g[q];
    }
    lam_out[row] = lam[row] + dl;
    if (Q) r[row] -= dr;
}

void launch_update_lr(int n, int k, const double* W, const double* Q, const double* g, double* lam, double* r,
                      hipStream_t st, double* lam_out) {
    if (!n) return;
    if (!lam_out) lam_out = lam;
    if (k == 64)
        k_update_lr64<<<(int)((16LL * n + 255) / 256), 256, 0, st>>>(n, W, Q, g, lam, lam_out, r, nullptr);
    else
        k_update_lr<<<(n + 255) / 256, 256, 0, st>>>(n, k, W, Q, g, lam, lam_out, r);
}

__global__ void __launch_bounds__(1024) k_colsum64(int nchunk, const double* __restrict__ part, double* __restrict__ out);

void launch_gemv_t(int n, int k, const double* A, const double* x, double* part, double* out, hipStream_t st) {
    if (k != 64) throw std::invalid_argument("launch_gemv_t takes 64 columns");
    // at least 64 rows per workgroup, up to 256 workgroups (one per CU)
    const int nchunk = std::max(1, std::min(256, (n + 63) / 64));
    k_gemv_t64<<<nchunk, 256, 0, st>>>(n, A, x, part);
    k_colsum64<<<1, 1024, 0, st>>>(nchunk, part, out);
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

// *out = sum of part[0..n) in a fixed order: 256 strided partial sums, then a fixed tree
__global__ void __launch_bounds__(256) k_sum(int n, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double red[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += part[i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// out[e] = sum_c part[c*64 + e] for e < 64: sixteen wavefronts take c = w mod 16, each with four
// running sums (c = w + 16(4i + u), sum u) so that four loads are in flight; fixed-order combine
__global__ void __launch_bounds__(1024) k_colsum64(int nchunk, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double red[16][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = wave; c < nchunk; c += 64)
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c + 16 * u < nchunk) v[u] += part[(long long)(c + 16 * u) * 64 + lane];
    red[wave][lane] = (v[0] + v[1]) + (v[2] + v[3]);
    __syncthreads();
    if (wave == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < 16; ++w) t += red[w][lane];
        out[lane] = t;
    }
}

void launch_rowsum_dot(int n, int k, const double* r, const double* Z, double* part, double* out, hipStream_t st) {
    const int nb = k == 64 ? std::max(1, std::min(1024, (n + 63) / 64)) : std::max(1, std::min(256, (n + 255) / 256));
    if (k == 64)
        k_rowsum_dot64<<<nb, 256, 0, st>>>(n, r, Z, part);
    else
        k_rowsum_dot<<<nb, 256, 0, st>>>(n, k, r, Z, part);
    k_sum<<<1, 256, 0, st>>>(nb, part, out);
}

// part[blk] = sum of (a - b)^2, part[256 + blk] = sum of b^2 over the workgroup's grid-stride
// share of the len entries (fixed order within the workgroup)
__global__ void __launch_bounds__(256) k_diff_norms(long long len, const double* __restrict__ a,
                                                    const double* __restrict__ b, double* __restrict__ part) {
    __shared__ double red[2][4];
    double d2 = 0.0, b2 = 0.0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < len; i += 256LL * gridDim.x) {
        const double bv = b[i], dv = a[i] - bv;
        d2 = fma(dv, dv, d2);
        b2 = fma(bv, bv, b2);
    }
    d2 = warp_sum(d2);
    b2 = warp_sum(b2);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = d2;
        red[1][threadIdx.x >> 6] = b2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[blockIdx.x] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        part[256 + blockIdx.x] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

void launch_diff_norms(long long len, const double* a, const double* b, double* part, double* out, hipStream_t st) {
    const int nb = (int)std::max(1LL, std::min(256LL, (len + 255) / 256));
    k_diff_norms<<<nb, 256, 0, st>>>(len, a, b, part);
    k_sum<<<1, 256, 0, st>>>(nb, part, out);
    k_sum<<<1, 256, 0, st>>>(nb, part + 256, out + 1);
}

// out[d] = sum over the rows of design d of r[row] * sum_c Z[row][c]; one workgroup per design,
// fixed order (thread-strided partial sums, then a fixed tree)
// out[d] = r_d^T (Z_d 1) over design d's rows [seg[2d], seg[2d] + seg[2d+1]): kSegDotSplit
// workgroups per design, each over a contiguous slice of its rows (k = 64: wavefront per row,
// lane per column, coalesced; otherwise thread per row), then the slices in order.
constexpr int kSegDotSplit = 8;
__global__ void __launch_bounds__(256) k_seg_dot(const int* __restrict__ seg, int k, const double* __restrict__ r,
                                                 const double* __restrict__ Z, double* __restrict__ part) {
    __shared__ double red[4];
    const int d = blockIdx.y, sp = blockIdx.x, r0 = seg[2 * d], nr = seg[2 * d + 1];
    const int i0 = (int)((long long)nr * sp / kSegDotSplit), i1 = (int)((long long)nr * (sp + 1) / kSegDotSplit);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    double v = 0.0;
    if (k == 64) {
#pragma unroll 4
        for (int i = i0 + wave; i < i1; i += 4) {
            const long long row = r0 + i;
            v = fma(Z[row * 64 + lane], r[row], v);
        }
    } else {
        for (int i = i0 + tid; i < i1; i += 256) {
            const long long row = r0 + i;
            double z = 0.0;
            for (int c = 0; c < k; ++c) z += Z[row * k + c];
            v = fma(r[row], z, v);
        }
    }
    v = wave_sum_dpp(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (tid == 0) part[d * kSegDotSplit + sp] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_seg_dot_sum(int nseg, const double* __restrict__ part, double* __restrict__ out) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= nseg) return;
    double v = 0.0;
#pragma unroll
    for (int sp = 0; sp < kSegDotSplit; ++sp) v += part[d * kSegDotSplit + sp];
    out[d] = v;
}

void launch_seg_dot(const DevTopo& t, int k, const double* r, const double* Z, double* part, double* out,
                    hipStream_t st) {
    const int nseg = (int)t.dsg.size();
    if (nseg <= 1) return;
    k_seg_dot<<<dim3(kSegDotSplit, nseg), 256, 0, st>>>(t.seg, k, r, Z, part);
    k_seg_dot_sum<<<(nseg + 63) / 64, 64, 0, st>>>(nseg, part, out);
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
