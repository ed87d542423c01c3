// Solve-phase kernels: distribution of the load to the subdomains, the right-hand sides
// of the dual problems (Sec. 2.1 Eq. 7: d = B K^+ f - c, e = -R^T f; Sec. 2.2 Eq. 12:
// d_r, fbar_c), recovery of the primal solution, averaging of the subdomain copies and
// the compliance with its adjoint gradient.
#include "kernels.hpp"

#include <stdexcept>
#include "dense_wg.hpp"

namespace feti {

// f^s: a global load entry goes to the lowest-numbered subdomain holding its DOF.
__global__ void k_scatter_f(const SubMeta* __restrict__ subs, const int8_t* __restrict__ lcls,
                            const int* __restrict__ lidx, const int* __restrict__ lglob,
                            const int8_t* __restrict__ lown, const double* __restrict__ f, double* fi, double* fbeta) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= M.n_loc) return;
    const long long q = M.off_loc + l;
    const double v = lown[q] ? f[lglob[q]] : 0.0;
    const long long ob = M.off_b + M.off_c;
    switch (lcls[q]) {
        case CLS_I: fi[M.off_i + lidx[q]] = v; break;
        case CLS_B: fbeta[ob + lidx[q]] = v; break;
        case CLS_C: fbeta[ob + M.n_b + lidx[q]] = v; break;
        default: break;
    }
}

void launch_scatter_f(const DevTopo& t, const double* f, double* fi, double* fbeta, hipStream_t st) {
    k_scatter_f<<<dim3((t.max_nloc + 255) / 256, t.n_sub), 256, 0, st>>>(t.subs, t.lcls, t.lidx, t.lglob, t.lown, f,
                                                                         fi, fbeta);
}

// h <- L^{-1} h for the block-tridiagonal factor, one wavefront per subdomain.
__global__ void __launch_bounds__(64) k_bt_fsolve1(const SubMeta* __restrict__ subs, const LineMeta* __restrict__ lines,
                                                   const double* __restrict__ Lbuf, double* h) {
    extern __shared__ double xs[];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    const int lane = threadIdx.x;
    double* hs = h + M.off_i;
    for (int k = 0; k < M.n_lines; ++k) {
        const LineMeta Lk = lines[M.line0 + k];
        if (Lk.n == 0) continue;
        for (int r = lane; r < Lk.n; r += 64) {
            double v = hs[Lk.i0 + r];
            const double* Ls = Lbuf + Lk.off_sub + (long long)r * Lk.n_prev;
            for (int q = 0; q < Lk.n_prev; ++q) v -= Ls[q] * hs[Lk.i0 - Lk.n_prev + q];
            xs[r] = v;
        }
        __syncthreads();
        const double* D = Lbuf + Lk.off_diag;
        for (int r = 0; r < Lk.n; ++r) {
            const double xr = xs[r] / D[(long long)r * Lk.n + r];
            __syncthreads();
            if (lane == 0) xs[r] = xr;
            for (int q = r + 1 + lane; q < Lk.n; q += 64) xs[q] -= D[(long long)q * Lk.n + r] * xr;
            __syncthreads();
        }
        for (int r = lane; r < Lk.n; r += 64) hs[Lk.i0 + r] = xs[r];
        __syncthreads();
    }
}

// x <- L^{-T} x (backward, block upper-bidiagonal L^T), one wavefront per subdomain.
__global__ void __launch_bounds__(64) k_bt_bsolve1(const SubMeta* __restrict__ subs, const LineMeta* __restrict__ lines,
                                                   const double* __restrict__ Lbuf, double* x) {
    extern __shared__ double xs[];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    const int lane = threadIdx.x;
    double* xg = x + M.off_i;
    for (int k = M.n_lines - 1; k >= 0; --k) {
        const LineMeta Lk = lines[M.line0 + k];
        if (Lk.n == 0) continue;
        // t_k -= L_{k+1,k}^T x_{k+1}
        LineMeta Ln;
        Ln.n = 0;
        if (k + 1 < M.n_lines) Ln = lines[M.line0 + k + 1];
        for (int q = lane; q < Lk.n; q += 64) {
            double v = xg[Lk.i0 + q];
            if (Ln.n > 0) {
                const double* Ls = Lbuf + Ln.off_sub;
                for (int r = 0; r < Ln.n; ++r) v -= Ls[(long long)r * Lk.n + q] * xg[Ln.i0 + r];
            }
            xs[q] = v;
        }
        __syncthreads();
        const double* D = Lbuf + Lk.off_diag;
        for (int r = Lk.n - 1; r >= 0; --r) {
            const double xr = xs[r] / D[(long long)r * Lk.n + r];
            __syncthreads();
            if (lane == 0) xs[r] = xr;
            for (int q = lane; q < r; q += 64) xs[q] -= D[(long long)r * Lk.n + q] * xr;
            __syncthreads();
        }
        for (int q = lane; q < Lk.n; q += 64) xg[Lk.i0 + q] = xs[q];
        __syncthreads();
    }
}

// Sweeps with the explicit diagonal inverses (every line <= kSweepMaxLine DOFs): per line
// one product with the coupling block and one with L_kk^{-1}. One 1024-thread workgroup per
// subdomain: wavefront w takes rows w, w + 16, ... of a block and lane l its columns l and
// l + 64, so every load reads 512 contiguous bytes of a row, and all sixteen loads of a lane
// are in flight before the first is used. L_kk^{-1} is lower triangular: its zero upper part
// is not read. The forward sweep sums each row over its wavefront; the backward sweep (the
// transposed products) keeps per-lane column sums and adds the sixteen wavefronts' sums in
// LDS in a fixed order.
constexpr int kSwW = 16, kSwT = 64 * kSwW, kSwP = kSweepMaxLine / kSwW;   // rows per wavefront

// a[p][h] = A[w + 16 p][l + 64 h] (rows < nr, columns < nc and <= row when lower), 0 elsewhere
__device__ __forceinline__ void sweep_load(double (&a)[kSwP][2], const double* __restrict__ A, int nr, int nc,
                                           bool lower) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int p = 0; p < kSwP; ++p)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = w + kSwW * p, q = l + 64 * h;
            a[p][h] = (r < nr && q < nc && (!lower || q <= r)) ? A[(long long)r * nc + q] : 0.0;
        }
}

// y[r] = sum_q A[r][q] x[q] for the rows of this wavefront (result valid in every lane)
__device__ __forceinline__ void sweep_rows(const double (&a)[kSwP][2], const double* x, double (&y)[kSwP]) {
    const int l = threadIdx.x & 63;
    const double x0 = x[l], x1 = x[l + 64];
#pragma unroll
    for (int p = 0; p < kSwP; ++p) y[p] = wave_sum_dpp(a[p][0] * x0 + a[p][1] * x1);
}

// y[q] = sum_r A[r][q] x[r] over all rows (red: kSwW x 128 doubles of LDS; y in LDS, size 128)
__device__ __forceinline__ void sweep_cols(const double (&a)[kSwP][2], const double* x, double* red, double* y,
                                           int nc) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double c0 = 0.0, c1 = 0.0;
#pragma unroll
    for (int p = 0; p < kSwP; ++p) {
        const double xr = x[w + kSwW * p];
        c0 = fma(a[p][0], xr, c0);
        c1 = fma(a[p][1], xr, c1);
    }
    red[w * kSweepMaxLine + l] = c0;
    red[w * kSweepMaxLine + l + 64] = c1;
    __syncthreads();
    if (threadIdx.x < kSweepMaxLine && (int)threadIdx.x < nc) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kSwW; ++q) t += red[q * kSweepMaxLine + threadIdx.x];
        y[threadIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kSwT) k_bt_fsweep(const SubMeta* __restrict__ subs, const LineMeta* __restrict__ lines,
                                                    const double* __restrict__ Lbuf, const double* __restrict__ Li,
                                                    double* h) {
    __shared__ double xp[kSweepMaxLine], v[kSweepMaxLine];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double* hs = h + M.off_i;
    if (threadIdx.x < kSweepMaxLine) xp[threadIdx.x] = 0.0;
    double a[kSwP][2], y[kSwP];
    for (int k = 0; k < M.n_lines; ++k) {
        const LineMeta Lk = lines[M.line0 + k];
        if (Lk.n == 0) continue;
        // v = b_k - L_{k,k-1} x_{k-1}
        sweep_load(a, Lbuf + Lk.off_sub, Lk.n, Lk.n_prev, false);
        __syncthreads();   // xp of the previous line complete
        sweep_rows(a, xp, y);
#pragma unroll
        for (int p = 0; p < kSwP; ++p) {
            const int r = w + kSwW * p;
            if (l == 0 && r < Lk.n) v[r] = hs[Lk.i0 + r] - y[p];
        }
        if (threadIdx.x >= (unsigned)Lk.n && threadIdx.x < kSweepMaxLine) v[threadIdx.x] = 0.0;
        // x_k = L_kk^{-1} v
        sweep_load(a, Li + Lk.off_inv, Lk.n, Lk.n, true);
        __syncthreads();   // v complete, xp free
        sweep_rows(a, v, y);
#pragma unroll
        for (int p = 0; p < kSwP; ++p) {
            const int r = w + kSwW * p;
            if (l == 0 && r < Lk.n) {
                hs[Lk.i0 + r] = y[p];
                xp[r] = y[p];
            }
        }
        if (threadIdx.x >= (unsigned)Lk.n && threadIdx.x < kSweepMaxLine) xp[threadIdx.x] = 0.0;
    }
}

__global__ void __launch_bounds__(kSwT) k_bt_bsweep(const SubMeta* __restrict__ subs, const LineMeta* __restrict__ lines,
                                                    const double* __restrict__ Lbuf, const double* __restrict__ Li,
                                                    double* x) {
    __shared__ double xn[kSweepMaxLine], wv[kSweepMaxLine], cs[kSweepMaxLine];
    __shared__ double red[kSwW * kSweepMaxLine];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    double* xg = x + M.off_i;
    if (threadIdx.x < kSweepMaxLine) xn[threadIdx.x] = 0.0;
    double a[kSwP][2];
    for (int k = M.n_lines - 1; k >= 0; --k) {
        const LineMeta Lk = lines[M.line0 + k];
        if (Lk.n == 0) continue;
        // w = t_k - L_{k+1,k}^T x_{k+1}  (L_{k+1,k}: n_next x n, row-major)
        const int n_next = k + 1 < M.n_lines ? lines[M.line0 + k + 1].n : 0;
        const long long off_c = n_next > 0 ? lines[M.line0 + k + 1].off_sub : 0;
        sweep_load(a, Lbuf + off_c, n_next, Lk.n, false);
        __syncthreads();   // xn of the previous line complete, red free
        sweep_cols(a, xn, red, cs, Lk.n);
        __syncthreads();   // cs complete
        if (threadIdx.x < (unsigned)Lk.n) wv[threadIdx.x] = xg[Lk.i0 + threadIdx.x] - cs[threadIdx.x];
        else if (threadIdx.x < kSweepMaxLine) wv[threadIdx.x] = 0.0;
        // x_k = L_kk^{-T} w: x_q = sum_{r >= q} Li[r][q] w_r
        sweep_load(a, Li + Lk.off_inv, Lk.n, Lk.n, true);
        __syncthreads();   // wv complete, red free
        sweep_cols(a, wv, red, cs, Lk.n);
        __syncthreads();   // cs complete
        if (threadIdx.x < (unsigned)Lk.n) {
            xg[Lk.i0 + threadIdx.x] = cs[threadIdx.x];
            xn[threadIdx.x] = cs[threadIdx.x];
        } else if (threadIdx.x < kSweepMaxLine) {
            xn[threadIdx.x] = 0.0;
        }
    }
}

// Sweeps for lines of up to kSweepBigLine DOFs (3D plane blocks), on the same 1024-thread
// layout over 128 x 128 tiles: a tile's sixteen loads per lane are in flight together, the
// forward sweep accumulates a row tile over its column tiles before one wavefront sum per row,
// the backward sweep a column tile over its row tiles before one LDS reduction; the zero tiles
// above the diagonal of L_kk^{-1} are skipped.

// a[p][h] = A[r0 + w + 16 p][c0 + l + 64 h] (row-major, ld columns; rows < nr, columns < nc and,
// when lower, column <= row), 0 elsewhere
__device__ __forceinline__ void sweep_tile(double (&a)[kSwP][2], const double* __restrict__ A, int ld, int r0, int c0,
                                           int nr, int nc, bool lower) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int p = 0; p < kSwP; ++p)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = r0 + w + kSwW * p, q = c0 + l + 64 * h;
            a[p][h] = (r < nr && q < nc && (!lower || q <= r)) ? A[(long long)r * ld + q] : 0.0;
        }
}

// y[r] = sum_q A[r][q] x[q] for the rows of row tile rt (all column tiles), valid in every lane
__device__ __forceinline__ void big_rows(const double* __restrict__ A, int n, int nc, int rt, const double* x, bool lower,
                                         double (&y)[kSwP]) {
    const int l = threadIdx.x & 63;
    double part[kSwP];
#pragma unroll
    for (int p = 0; p < kSwP; ++p) part[p] = 0.0;
    const int ct_end = lower ? rt + 1 : (nc + kSweepMaxLine - 1) / kSweepMaxLine;
    for (int ct = 0; ct < ct_end; ++ct) {
        double a[kSwP][2];
        sweep_tile(a, A, nc, rt * kSweepMaxLine, ct * kSweepMaxLine, n, nc, lower);
        const double x0 = x[ct * kSweepMaxLine + l], x1 = x[ct * kSweepMaxLine + l + 64];
#pragma unroll
        for (int p = 0; p < kSwP; ++p) part[p] = fma(a[p][1], x1, fma(a[p][0], x0, part[p]));
    }
#pragma unroll
    for (int p = 0; p < kSwP; ++p) y[p] = wave_sum_dpp(part[p]);
}

// y[ct*128 + t] = sum_r A[r][ct*128 + t] x[r] over the rows r >= row of the diagonal when lower
// (red: kSwW x 128 doubles; y written by threads < 128; ends with a barrier)
__device__ __forceinline__ void big_cols(const double* __restrict__ A, int nr, int nc, int ct, const double* x,
                                         bool lower, double* red, double* y) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double c0 = 0.0, c1 = 0.0;
    const int rt_end = (nr + kSweepMaxLine - 1) / kSweepMaxLine;
    for (int rt = lower ? ct : 0; rt < rt_end; ++rt) {
        double a[kSwP][2];
        sweep_tile(a, A, nc, rt * kSweepMaxLine, ct * kSweepMaxLine, nr, nc, lower);
#pragma unroll
        for (int p = 0; p < kSwP; ++p) {
            const double xr = x[rt * kSweepMaxLine + w + kSwW * p];
            c0 = fma(a[p][0], xr, c0);
            c1 = fma(a[p][1], xr, c1);
        }
    }
    red[w * kSweepMaxLine + l] = c0;
    red[w * kSweepMaxLine + l + 64] = c1;
    __syncthreads();
    if (threadIdx.x < kSweepMaxLine) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kSwW; ++q) t += red[q * kSweepMaxLine + threadIdx.x];
        y[ct * kSweepMaxLine + threadIdx.x] = t;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kSwT) k_bt_fsweep_big(const SubMeta* __restrict__ subs,
                                                        const LineMeta* __restrict__ lines,
                                                        const double* __restrict__ Lbuf, const double* __restrict__ Li,
                                                        double* h) {
    __shared__ double xp[kSweepBigLine], v[kSweepBigLine];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double* hs = h + M.off_i;
    for (int q = threadIdx.x; q < kSweepBigLine; q += kSwT) xp[q] = 0.0;
    double y[kSwP];
    for (int k = 0; k < M.n_lines; ++k) {
        const LineMeta Lk = lines[M.line0 + k];
        if (Lk.n == 0) continue;
        const int nt = (Lk.n + kSweepMaxLine - 1) / kSweepMaxLine;
        __syncthreads();   // xp of the previous line complete
        // v = b_k - L_{k,k-1} x_{k-1}
        for (int rt = 0; rt < nt; ++rt) {
            if (Lk.n_prev > 0) {
                big_rows(Lbuf + Lk.off_sub, Lk.n, Lk.n_prev, rt, xp, false, y);
            } else {
#pragma unroll
                for (int p = 0; p < kSwP; ++p) y[p] = 0.0;
            }
#pragma unroll
            for (int p = 0; p < kSwP; ++p) {
                const int r = rt * kSweepMaxLine + w + kSwW * p;
                if (l == 0 && r < Lk.n) v[r] = hs[Lk.i0 + r] - y[p];
            }
        }
        for (int q = Lk.n + threadIdx.x; q < kSweepBigLine; q += kSwT) v[q] = 0.0;
        __syncthreads();   // v complete, xp free
        // x_k = L_kk^{-1} v
        for (int rt = 0; rt < nt; ++rt) {
            big_rows(Li + Lk.off_inv, Lk.n, Lk.n, rt, v, true, y);
#pragma unroll
            for (int p = 0; p < kSwP; ++p) {
                const int r = rt * kSweepMaxLine + w + kSwW * p;
                if (l == 0 && r < Lk.n) {
                    hs[Lk.i0 + r] = y[p];
                    xp[r] = y[p];
                }
            }
        }
        for (int q = Lk.n + threadIdx.x; q < kSweepBigLine; q += kSwT) xp[q] = 0.0;
    }
}

__global__ void __launch_bounds__(kSwT) k_bt_bsweep_big(const SubMeta* __restrict__ subs,
                                                        const LineMeta* __restrict__ lines,
                                                        const double* __restrict__ Lbuf, const double* __restrict__ Li,
                                                        double* x) {
    __shared__ double xn[kSweepBigLine], wv[kSweepBigLine], cs[kSweepBigLine];
    __shared__ double red[kSwW * kSweepMaxLine];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    double* xg = x + M.off_i;
    for (int q = threadIdx.x; q < kSweepBigLine; q += kSwT) xn[q] = 0.0;
    for (int k = M.n_lines - 1; k >= 0; --k) {
        const LineMeta Lk = lines[M.line0 + k];
        if (Lk.n == 0) continue;
        const int nt = (Lk.n + kSweepMaxLine - 1) / kSweepMaxLine;
        // w = t_k - L_{k+1,k}^T x_{k+1}  (L_{k+1,k}: n_next x n, row-major)
        const int n_next = k + 1 < M.n_lines ? lines[M.line0 + k + 1].n : 0;
        __syncthreads();   // xn of the previous line complete
        if (n_next > 0) {
            const double* C = Lbuf + lines[M.line0 + k + 1].off_sub;
            for (int ct = 0; ct < nt; ++ct) big_cols(C, n_next, Lk.n, ct, xn, false, red, cs);
        }
        for (int q = threadIdx.x; q < kSweepBigLine; q += kSwT)
            wv[q] = q < Lk.n ? xg[Lk.i0 + q] - (n_next > 0 ? cs[q] : 0.0) : 0.0;
        __syncthreads();   // wv complete
        // x_k = L_kk^{-T} w: x_q = sum_{r >= q} Li[r][q] w_r
        for (int ct = 0; ct < nt; ++ct) big_cols(Li + Lk.off_inv, Lk.n, Lk.n, ct, wv, true, red, cs);
        for (int q = threadIdx.x; q < kSweepBigLine; q += kSwT) {
            if (q < Lk.n) {
                xg[Lk.i0 + q] = cs[q];
                xn[q] = cs[q];
            } else {
                xn[q] = 0.0;
            }
        }
    }
}

// Li = L_kk^{-1} for every line block of every subdomain (identity, then L_kk^{-1} I).
__global__ void __launch_bounds__(256) k_bt_invert(const LineMeta* __restrict__ lines, const double* __restrict__ Lbuf,
                                                   double* Li) {
    __shared__ double lds[kLdsDoubles];
    const LineMeta Lk = lines[blockIdx.x];
    if (Lk.n == 0) return;
    double* X = Li + Lk.off_inv;
    for (int e = threadIdx.x; e < Lk.n * Lk.n; e += 256) X[e] = (e / Lk.n == e % Lk.n) ? 1.0 : 0.0;
    __syncthreads();
    wg_trsm_lower(Lk.n, Lk.n, Lbuf + Lk.off_diag, Lk.n, X, Lk.n, 1, lds);
}

// (lines <= 128 DOFs get their inverses from the factorisation itself; longer lines, up to
// kSweepBigLine, from this kernel)
void launch_bt_invert(const DevTopo& t, const double* L, double* Li, hipStream_t st) {
    if (t.max_line > kSweepMaxLine && t.max_line <= kSweepBigLine && t.n_lines_tot > 0)
        k_bt_invert<<<t.n_lines_tot, 256, 0, st>>>(t.lines, L, Li);
}

void launch_bt_fsolve1(const DevTopo& t, const double* L, const double* Li, double* h, hipStream_t st) {
    if (t.max_line <= kSweepMaxLine)
        k_bt_fsweep<<<t.n_sub, kSwT, 0, st>>>(t.subs, t.lines, L, Li, h);
    else if (t.max_line <= kSweepBigLine)
        k_bt_fsweep_big<<<t.n_sub, kSwT, 0, st>>>(t.subs, t.lines, L, Li, h);
    else
        k_bt_fsolve1<<<t.n_sub, 64, sizeof(double) * std::max(1, t.max_line), st>>>(t.subs, t.lines, L, h);
}

void launch_bt_bsolve1(const DevTopo& t, const double* L, const double* Li, double* x, hipStream_t st) {
    if (t.max_line <= kSweepMaxLine)
        k_bt_bsweep<<<t.n_sub, kSwT, 0, st>>>(t.subs, t.lines, L, Li, x);
    else if (t.max_line <= kSweepBigLine)
        k_bt_bsweep_big<<<t.n_sub, kSwT, 0, st>>>(t.subs, t.lines, L, Li, x);
    else
        k_bt_bsolve1<<<t.n_sub, 64, sizeof(double) * std::max(1, t.max_line), st>>>(t.subs, t.lines, L, x);
}

// g = fbeta - Z^T h in two passes. Pass 1: workgroup (slice sp, subdomain s) sums rows
// [i0, i1) of Z_s (n_i / kZtSplit each) for every column (thread = columns j, j + 256, ...),
// eight rows in flight, into part[sp * stride + ob + j]; each workgroup streams one contiguous
// block of Z_s. Pass 2 adds the slices in order (deterministic).
constexpr int kZtSplit = 8;
__global__ void __launch_bounds__(256) k_zt_part(const SubMeta* __restrict__ subs, const double* __restrict__ Z,
                                                 const double* __restrict__ h, double* __restrict__ part,
                                                 long long stride) {
    const int s = blockIdx.y, sp = blockIdx.x;
    const SubMeta M = subs[s];
    const int i0 = (int)((long long)M.n_i * sp / kZtSplit), i1 = (int)((long long)M.n_i * (sp + 1) / kZtSplit);
    const long long ob = M.off_b + M.off_c;
    const double* hs = h + M.off_i;
    for (int j = threadIdx.x; j < M.n_beta; j += 256) {
        const double* Zc = Z + M.off_Z + j;
        double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int i = i0;
        for (; i + 8 <= i1; i += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = fma(Zc[(long long)(i + u) * M.n_beta], hs[i + u], v[u]);
        }
        for (int u = 0; i < i1; ++i, ++u) v[u] = fma(Zc[(long long)i * M.n_beta], hs[i], v[u]);
        part[sp * stride + ob + j] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
}

__global__ void k_zt_sum(const SubMeta* __restrict__ subs, const double* __restrict__ part, long long stride,
                         const double* __restrict__ fbeta, double* __restrict__ g) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M.n_beta) return;
    const long long ob = M.off_b + M.off_c;
    double v = 0.0;
#pragma unroll
    for (int sp = 0; sp < kZtSplit; ++sp) v += part[sp * stride + ob + j];
    g[ob + j] = fbeta[ob + j] - v;
}

void launch_zt_gemv(const DevTopo& t, const double* Z, const double* h, const double* fbeta, double* g, double* part,
                    hipStream_t st) {
    const long long stride = t.nb_tot + t.nc_tot;
    if (kZtSplit * stride > kGramPartCap) throw std::length_error("Z^T h partial buffer too small");
    k_zt_part<<<dim3(kZtSplit, t.n_sub), 256, 0, st>>>(t.subs, Z, h, part, stride);
    k_zt_sum<<<dim3((t.max_beta + 255) / 256, t.n_sub), 256, 0, st>>>(t.subs, part, stride, fbeta, g);
}

// x = h - Z ubeta: wavefront per four interior rows (their loads in flight together), each row
// reduced over the wavefront
constexpr int kZRows = 4;
__global__ void __launch_bounds__(256) k_z_gemv(const SubMeta* __restrict__ subs, const double* __restrict__ Z,
                                                const double* __restrict__ ubeta, const double* __restrict__ h,
                                                double* x) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int i0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * kZRows, lane = threadIdx.x & 63;
    if (i0 >= M.n_i) return;
    const long long ob = M.off_b + M.off_c;
    double v[kZRows];
#pragma unroll
    for (int r = 0; r < kZRows; ++r) v[r] = 0.0;
    for (int j = lane; j < M.n_beta; j += 64) {
        const double u = ubeta[ob + j];
#pragma unroll
        for (int r = 0; r < kZRows; ++r) {
            const int i = min(i0 + r, M.n_i - 1);
            v[r] = fma(Z[M.off_Z + (long long)i * M.n_beta + j], u, v[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < kZRows; ++r) {
        const double t = wave_sum_dpp(v[r]);
        if (lane == 0 && i0 + r < M.n_i) x[M.off_i + i0 + r] = h[M.off_i + i0 + r] - t;
    }
}

void launch_z_gemv(const DevTopo& t, const double* Z, const double* ubeta, const double* h, double* x,
                   hipStream_t st) {
    k_z_gemv<<<dim3((t.max_ni + 4 * kZRows - 1) / (4 * kZRows), t.n_sub), 256, 0, st>>>(t.subs, Z, ubeta, h, x);
}

// y = [F_s; F_rc^sT] g_b (FP64), wavefront per row
__global__ void __launch_bounds__(256) k_local_F(const SubMeta* __restrict__ subs, const double* __restrict__ F64,
                                                 const double* __restrict__ g, double* yb, double* yc) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= M.n_b + M.n_c) return;
    const long long ob = M.off_b + M.off_c;
    const int prow = row < M.n_b ? row : M.rowT + row - M.n_b;   // physical row of F_rc^T entries
    const double* Fr = F64 + M.off_F + (long long)prow * M.ldF;
    double v = 0.0;
    for (int j = lane; j < M.n_b; j += 64) v += Fr[j] * g[ob + j];
    v = warp_sum(v);
    if (lane == 0) {
        if (row < M.n_b)
            yb[M.off_b + row] = v;
        else
            yc[M.off_c + row - M.n_b] = v;
    }
}

void launch_local_F(const DevTopo& t, const double* F64, const double* g, double* yb, double* yc, hipStream_t st) {
    k_local_F<<<dim3((t.max_nb + t.max_nc + 3) / 4, t.n_sub), 256, 0, st>>>(t.subs, F64, g, yb, yc);
}

// fbar_c^s = g_c - F_rc^sT g_b   (the local reduced corner load)
__global__ void k_fbar(const SubMeta* __restrict__ subs, int n_sub, const double* __restrict__ g,
                       const double* __restrict__ yc, double* fbar_s) {
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    for (int c = threadIdx.x; c < M.n_c; c += blockDim.x)
        fbar_s[M.off_c + c] = g[M.off_b + M.off_c + M.n_b + c] - yc[M.off_c + c];
}

void launch_fbar(const DevTopo& t, const double* g, const double* yc, double* fbar_s, hipStream_t st) {
    k_fbar<<<t.n_sub, 64, 0, st>>>(t.subs, t.n_sub, g, yc, fbar_s);
}

// xb = B^sT lambda for every interface DOF
__global__ void k_gather_B(long long nb_tot, const int* __restrict__ bg_ptr, const int* __restrict__ bg_row,
                           const int8_t* __restrict__ bg_sg, const double* __restrict__ lam, double* xb) {
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= nb_tot) return;
    double v = 0.0;
    for (int e = bg_ptr[q]; e < bg_ptr[q + 1]; ++e) v += bg_sg[e] * lam[bg_row[e]];
    xb[q] = v;
}

void launch_gather_B(const DevTopo& t, const double* lam, double* xb, hipStream_t st) {
    if (t.nb_tot) k_gather_B<<<(int)((t.nb_tot + 255) / 256), 256, 0, st>>>(t.nb_tot, t.bg_ptr, t.bg_row, t.bg_sg, lam, xb);
}

// Interface displacements of the recovery: u_b = F_s (g_b - S_bc u_c^s - (B^sT lambda)_b) and
// u_beta = [u_b; u_c^s] (FETI-DP; in TFETI n_c = 0 and F_s is the pseudo-inverse block), in two
// passes. k_ub_rhs: gh_s = g_b - x_b - S_bc u_c (thread per interface row, x_b = (B^sT lambda)_b)
// into scratch indexed like x_b. k_ub_gemv: u_b = F_s gh_s, a wavefront per row and 16 rows per
// workgroup (many workgroups per subdomain), then the corner values behind the interface rows.
__global__ void __launch_bounds__(256) k_ub_rhs(const SubMeta* __restrict__ subs, const double* __restrict__ S,
                                                const double* __restrict__ g, const double* __restrict__ xb,
                                                const double* __restrict__ uc, const int* __restrict__ c_glob,
                                                double* __restrict__ gh) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M.n_b) return;
    const long long ob = M.off_b + M.off_c;
    double v = g[ob + j] - xb[M.off_b + j];
    if (S)
        for (int c = 0; c < M.n_c; ++c)
            v -= S[M.off_S + (long long)j * M.n_beta + M.n_b + c] * uc[c_glob[M.off_c + c]];
    gh[M.off_b + j] = v;
}

constexpr int kUbRows = 16;
__global__ void __launch_bounds__(256) k_ub_gemv(const SubMeta* __restrict__ subs, const double* __restrict__ F64,
                                                 const double* __restrict__ gh, const double* __restrict__ uc,
                                                 const int* __restrict__ c_glob, double* __restrict__ ubeta) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long ob = M.off_b + M.off_c;
    const double* gs = gh + M.off_b;
    for (int rr = wave; rr < kUbRows; rr += 4) {
        const int row = blockIdx.x * kUbRows + rr;
        if (row >= M.n_b) break;   // uniform over the wavefront
        const double* Fr = F64 + M.off_F + (long long)row * M.ldF;
        double v0 = 0.0, v1 = 0.0;
        int j = lane;
        for (; j + 64 < M.n_b; j += 128) {
            v0 = fma(Fr[j], gs[j], v0);
            v1 = fma(Fr[j + 64], gs[j + 64], v1);
        }
        if (j < M.n_b) v0 = fma(Fr[j], gs[j], v0);
        const double v = wave_sum_dpp(v0 + v1);
        if (lane == 0) ubeta[ob + row] = v;
    }
    if (blockIdx.x == 0 && uc)
        for (int c = threadIdx.x; c < M.n_c; c += 256) ubeta[ob + M.n_b + c] = uc[c_glob[M.off_c + c]];
}

void launch_dp_ub(const DevTopo& t, const double* F64, const double* S, const double* g, const double* xb,
                  const double* uc, double* ubeta, double* scratch, hipStream_t st) {
    k_ub_rhs<<<dim3((t.max_nb + 255) / 256, t.n_sub), 256, 0, st>>>(t.subs, S, g, xb, uc, t.c_glob, scratch);
    k_ub_gemv<<<dim3((t.max_nb + kUbRows - 1) / kUbRows, t.n_sub), 256, 0, st>>>(t.subs, F64, scratch, uc, t.c_glob,
                                                                                ubeta);
}

void launch_tfeti_ub(const DevTopo& t, const double* F64, const double* g, const double* xb, double* ubeta,
                     double* scratch, hipStream_t st) {
    launch_dp_ub(t, F64, nullptr, g, xb, nullptr, ubeta, scratch, st);
}

// ---- rigid-body modes of a local DOF (same basis as the setup kernels) ----
__device__ inline void rbm_of_local(const SubMeta& M, int dim, int l, double* r) {
    const int node = l / dim, comp = l % dim;
    const int ix = node % M.nn[0], iy = (node / M.nn[0]) % M.nn[1], iz = node / (M.nn[0] * M.nn[1]);
    const double x = ix - 0.5 * (M.nn[0] - 1), y = iy - 0.5 * (M.nn[1] - 1), z = iz - 0.5 * (M.nn[2] - 1);
    const int nm = dim == 2 ? 3 : 6;
    for (int m = 0; m < nm; ++m) r[m] = 0.0;
    r[comp] = 1.0;
    if (dim == 2) {
        r[2] = comp == 0 ? -y : x;
    } else {
        r[3] = comp == 0 ? -y : (comp == 1 ? x : 0.0);
        r[4] = comp == 1 ? -z : (comp == 2 ? y : 0.0);
        r[5] = comp == 0 ? z : (comp == 2 ? -x : 0.0);
    }
}

// TFETI e_s = -Rhat_s^T f^s with Rhat_s = R_s C_s^{-T} over all local DOFs.
__global__ void __launch_bounds__(256) k_tfeti_e(const SubMeta* __restrict__ subs, int dim, const int8_t* __restrict__ lcls,
                                                 const int* __restrict__ lidx, const double* __restrict__ fi,
                                                 const double* __restrict__ fbeta, const double* __restrict__ Cit,
                                                 double* e) {
    __shared__ double red[256][6];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    const int nm = dim == 2 ? 3 : 6;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int l = threadIdx.x; l < M.n_loc; l += 256) {
        const long long q = M.off_loc + l;
        double f = 0.0;
        if (lcls[q] == CLS_I) f = fi[M.off_i + lidx[q]];
        else if (lcls[q] == CLS_B) f = fbeta[M.off_b + M.off_c + lidx[q]];
        if (f == 0.0) continue;
        double r[6];
        rbm_of_local(M, dim, l, r);
        for (int m = 0; m < nm; ++m) acc[m] += r[m] * f;
    }
    for (int m = 0; m < 6; ++m) red[threadIdx.x][m] = acc[m];
    __syncthreads();
    if (threadIdx.x < nm) {
        const int m = threadIdx.x;
        double tot[6];
        for (int a = 0; a < nm; ++a) {
            double v = 0.0;
            for (int u = 0; u < 256; ++u) v += red[u][a];
            tot[a] = v;
        }
        double v = 0.0;
        for (int a = 0; a < nm; ++a) v += tot[a] * Cit[s * 36 + a * nm + m];
        e[s * nm + m] = -v;
    }
}

void launch_tfeti_e(const DevTopo& t, const double* fi, const double* fbeta, const double* Cit, double* e,
                    hipStream_t st) {
    k_tfeti_e<<<t.n_sub, 256, 0, st>>>(t.subs, t.dim, t.lcls, t.lidx, fi, fbeta, Cit, e);
}

// Local displacement vector u^s (local DOF order) from its interior and interface parts,
// plus the rigid-body part Rhat_s alpha_s for TFETI.
__global__ void k_assemble_loc(const SubMeta* __restrict__ subs, int dim, const int8_t* __restrict__ lcls,
                               const int* __restrict__ lidx, const double* __restrict__ ui,
                               const double* __restrict__ ubeta, const double* __restrict__ Cit,
                               const double* __restrict__ alpha, double* uloc) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= M.n_loc) return;
    const long long q = M.off_loc + l;
    const long long ob = M.off_b + M.off_c;
    double v = 0.0;
    switch (lcls[q]) {
        case CLS_I: v = ui[M.off_i + lidx[q]]; break;
        case CLS_B: v = ubeta[ob + lidx[q]]; break;
        case CLS_C: v = ubeta[ob + M.n_b + lidx[q]]; break;
        default: v = 0.0; break;
    }
    if (alpha) {
        const int nm = dim == 2 ? 3 : 6;
        double r[6];
        rbm_of_local(M, dim, l, r);
        for (int m = 0; m < nm; ++m) {
            double rh = 0.0;
            for (int a = 0; a < nm; ++a) rh += r[a] * Cit[s * 36 + a * nm + m];
            v += rh * alpha[s * nm + m];
        }
    }
    uloc[q] = v;
}

void launch_assemble_loc(const DevTopo& t, const double* ui, const double* ubeta, const double* Cit,
                         const double* alpha, double* uloc, hipStream_t st) {
    k_assemble_loc<<<dim3((t.max_nloc + 255) / 256, t.n_sub), 256, 0, st>>>(t.subs, t.dim, t.lcls, t.lidx, ui, ubeta,
                                                                            Cit, alpha, uloc);
}

// Global u = average of the subdomain copies of every DOF.
__global__ void k_average(long long n_dof, int dim, int nx, int ny, int nsx, int nsy, const int* __restrict__ axf0,
                          const int* __restrict__ axc0, const int* __restrict__ axf1, const int* __restrict__ axc1,
                          const int* __restrict__ axf2, const int* __restrict__ axc2,
                          const SubMeta* __restrict__ subs, const double* __restrict__ uloc, double* u) {
    const long long gd = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (gd >= n_dof) return;
    const long long node = gd / dim;
    const int comp = (int)(gd % dim);
    const int x = (int)(node % (nx + 1));
    const int y = (int)((node / (nx + 1)) % (ny + 1));
    const int z = dim == 3 ? (int)(node / ((long long)(nx + 1) * (ny + 1))) : 0;
    double acc = 0.0;
    int cnt = 0;
    for (int kz = 0; kz < axc2[z]; ++kz)
        for (int ky = 0; ky < axc1[y]; ++ky)
            for (int kx = 0; kx < axc0[x]; ++kx) {
                const int s = (axf0[x] + kx) + nsx * ((axf1[y] + ky) + nsy * (axf2[z] + kz));
                const SubMeta& M = subs[s];
                const int ln = (x - M.lo[0]) + M.nn[0] * ((y - M.lo[1]) + M.nn[1] * (z - M.lo[2]));
                acc += uloc[M.off_loc + (long long)ln * dim + comp];
                ++cnt;
            }
    u[gd] = acc / cnt;
}

void launch_average(const DevTopo& t, const double* uloc, double* u, hipStream_t st) {
    // one launch per design: the subdomain of a node follows from that design's grid
    for (const DesignDev& D : t.dsg)
        if (D.n_dof)
            k_average<<<(int)((D.n_dof + 255) / 256), 256, 0, st>>>(
                D.n_dof, t.dim, D.nel[0], D.nel[1], D.nsub[0], D.nsub[1], D.axf[0], D.axc[0], D.axf[1], D.axc[1],
                D.axf[2], D.axc[2], t.subs + D.sub0, uloc, u + D.dof0);
}

// Compliance c = f^T u (two-stage reduction) and gradient
// dc/drho_e = -p rho_e^(p-1) (E0 - Emin) u_e^T K0 u_e (one thread per element).
__global__ void __launch_bounds__(256) k_dot_part(long long n, const double* __restrict__ a, const double* __restrict__ b,
                                                  double* part) {
    __shared__ double red[4];
    double v = 0.0;
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) v += a[i] * b[i];
    v = warp_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_sum_parts(int n, const double* __restrict__ part, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double v = 0.0;
        for (int i = 0; i < n; ++i) v += part[i];
        *out = v;
    }
}

__global__ void k_grad(long long n_el, int dim, int nx, int ny, const double* __restrict__ K0,
                       const double* __restrict__ u, const double* __restrict__ rho, double p, double E0, double Emin,
                       double* g) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= n_el) return;
    const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = dim == 3 ? (int)(e / ((long long)nx * ny)) : 0;
    const int ncorner = 1 << dim, ne = dim * ncorner;
    double ue[24];
    for (int a = 0; a < ncorner; ++a) {
        const int x = ex + (a & 1), y = ey + ((a >> 1) & 1), z = ez + ((a >> 2) & 1);
        const long long node = x + (long long)(nx + 1) * (y + (long long)(ny + 1) * z);
        for (int c = 0; c < dim; ++c) ue[a * dim + c] = u[node * dim + c];
    }
    double en = 0.0;
    for (int i = 0; i < ne; ++i) {
        double v = 0.0;
        for (int j = 0; j < ne; ++j) v += K0[i * ne + j] * ue[j];
        en += ue[i] * v;
    }
    g[e] = -p * pow(rho[e], p - 1.0) * (E0 - Emin) * en;
}

void launch_compliance(const DevTopo& t, const double* f, const double* u, const double* rho, double p, double E0,
                       double Emin, double* part, double* c, double* g, hipStream_t st) {
    // part must hold 256 doubles; t.K0dev holds the unit element matrix. One compliance c[d] and
    // one gradient block per design.
    for (size_t d = 0; d < t.dsg.size(); ++d) {
        const DesignDev& D = t.dsg[d];
        k_dot_part<<<256, 256, 0, st>>>(D.n_dof, f + D.dof0, u + D.dof0, part);
        k_sum_parts<<<1, 64, 0, st>>>(256, part, c + d);
        if (g && D.n_el)
            k_grad<<<(int)((D.n_el + 255) / 256), 256, 0, st>>>(D.n_el, t.dim, D.nel[0], D.nel[1], t.K0dev,
                                                                u + D.dof0, rho + D.el0, p, E0, Emin, g + D.el0);
    }
}

}  // namespace feti
