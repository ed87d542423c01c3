// Setup kernels: SIMP assembly of the subdomain stiffness blocks, block-tridiagonal
// Cholesky of the interior blocks, the interface Schur complement, explicit local dual
// operators F_s, preconditioner blocks, scaling weights and coarse matrices.
#include "dense_wg.hpp"
#include "kernels.hpp"

namespace feti {

// ---------------------------------------------------------------------------------------
// Assembly (Sec. 1 Eq. 1 and Sec. 2 Eq. 3): K^s = sum_e (Emin + rho_e^p (E0 - Emin)) K0.
// One thread per (subdomain, local node a); it forms every dpn x dpn block K_ab with its
// 3^dim neighbours b and routes each entry by the classes of its two DOFs:
//   (i, i) -> block-tridiagonal storage of K_ii (diagonal and sub-diagonal line blocks),
//   (i, beta) -> Z (becomes L^{-1} K_i,beta), (beta, beta) -> S (becomes the Schur complement),
//   diagonal -> diag (k-scaling). Each entry has exactly one writer: no atomics.
__global__ void k_assemble(const SubMeta* __restrict__ subs, const LineMeta* __restrict__ lines, int dim,
                           const double* __restrict__ K0, const double* __restrict__ Emod,
                           const int8_t* __restrict__ lcls, const int* __restrict__ lidx,
                           double* __restrict__ Lbuf, double* __restrict__ Zbuf, double* __restrict__ Sbuf,
                           double* __restrict__ diag) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int nnodes = M.nn[0] * M.nn[1] * M.nn[2];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nnodes) return;
    const int dpn = dim, ne = dpn << dim;  // element DOFs
    const int ax = a % M.nn[0], ay = (a / M.nn[0]) % M.nn[1], az = a / (M.nn[0] * M.nn[1]);
    const int ex_max = M.nn[0] - 1, ey_max = M.nn[1] - 1, ez_max = dim == 3 ? M.nn[2] - 1 : 1;
    const int zlo = dim == 3 ? -1 : 0, zhi = dim == 3 ? 1 : 0;
    const int line_a = dim == 2 ? ay : az;
    for (int dz = zlo; dz <= zhi; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int bx = ax + dx, by = ay + dy, bz = az + dz;
                if (bx < 0 || by < 0 || bz < 0 || bx >= M.nn[0] || by >= M.nn[1] || bz >= M.nn[2]) continue;
                const int b = bx + M.nn[0] * (by + M.nn[1] * bz);
                double blk[9];
                for (int q = 0; q < 9; ++q) blk[q] = 0.0;
                // elements containing both nodes
                const int ex0 = max(max(ax, bx) - 1, 0), ex1 = min(min(ax, bx), ex_max - 1);
                const int ey0 = max(max(ay, by) - 1, 0), ey1 = min(min(ay, by), ey_max - 1);
                const int ez0 = dim == 3 ? max(max(az, bz) - 1, 0) : 0;
                const int ez1 = dim == 3 ? min(min(az, bz), ez_max - 1) : 0;
                for (int ez = ez0; ez <= ez1; ++ez)
                    for (int ey = ey0; ey <= ey1; ++ey)
                        for (int ex = ex0; ex <= ex1; ++ex) {
                            const int ca = (ax - ex) + 2 * (ay - ey) + (dim == 3 ? 4 * (az - ez) : 0);
                            const int cb = (bx - ex) + 2 * (by - ey) + (dim == 3 ? 4 * (bz - ez) : 0);
                            const long long ge = M.el0 + (long long)(M.lo[0] + ex) +
                                                 (long long)M.nelx * ((M.lo[1] + ey) + (long long)M.nely * (M.lo[2] + ez));
                            const double E = Emod[ge];
                            for (int ci = 0; ci < dpn; ++ci)
                                for (int cj = 0; cj < dpn; ++cj)
                                    blk[ci * dpn + cj] += E * K0[(ca * dpn + ci) * ne + cb * dpn + cj];
                        }
                const int line_b = dim == 2 ? by : bz;
                for (int ci = 0; ci < dpn; ++ci) {
                    const long long pl = M.off_loc + (long long)a * dpn + ci;
                    const int cp = lcls[pl], ip = lidx[pl];
                    for (int cj = 0; cj < dpn; ++cj) {
                        const long long ql = M.off_loc + (long long)b * dpn + cj;
                        const double v = blk[ci * dpn + cj];
                        if (pl == ql) diag[pl] = v;
                        const int cq = lcls[ql], iq = lidx[ql];
                        if (cp == CLS_X || cq == CLS_X) continue;
                        if (cp == CLS_I) {
                            if (cq == CLS_I) {
                                const LineMeta La = lines[M.line0 + line_a];
                                if (line_a == line_b) {
                                    Lbuf[La.off_diag + (long long)(ip - La.i0) * La.n + (iq - La.i0)] = v;
                                } else if (line_b == line_a - 1) {
                                    const int i0b = La.i0 - La.n_prev;
                                    Lbuf[La.off_sub + (long long)(ip - La.i0) * La.n_prev + (iq - i0b)] = v;
                                }
                            } else {
                                const int jb = cq == CLS_B ? iq : M.n_b + iq;
                                Zbuf[M.off_Z + (long long)ip * M.n_beta + jb] = v;
                            }
                        } else if (cq != CLS_I) {
                            const int jp = cp == CLS_B ? ip : M.n_b + ip;
                            const int jq = cq == CLS_B ? iq : M.n_b + iq;
                            Sbuf[M.off_S + (long long)jp * M.n_beta + jq] = v;
                        }
                    }
                }
            }
}

// ---------------------------------------------------------------------------------------
// The interior-interface coupling blocks of K^s (Sec. 2, Eq. 3) applied without storing them:
// the entries are formed from the element densities exactly as in k_assemble (same element
// sums), one thread per (subdomain, local node a), only for node pairs (a, b) that carry the
// two classes:
//   to_beta = 0: out_i    = f_i    - K_i,beta in_beta  (rows: interior DOFs of a)
//   to_beta = 1: out_beta = f_beta - K_beta,i in_i     (rows: interface and corner DOFs of a)
// Interior vectors sit at off_i, beta vectors at off_b + off_c (interface DOFs, then corners).
__global__ void k_coupling(const SubMeta* __restrict__ subs, int dim, const double* __restrict__ K0,
                           const double* __restrict__ Emod, const int8_t* __restrict__ lcls, const int* __restrict__ lidx,
                           int to_beta, const double* __restrict__ in, const double* __restrict__ f,
                           double* __restrict__ out) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int nnodes = M.nn[0] * M.nn[1] * M.nn[2];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nnodes) return;
    const int dpn = dim, ne = dpn << dim;
    const long long ob = M.off_b + M.off_c;
    // row DOFs of a in the output class
    bool any_row = false;
    for (int ci = 0; ci < dpn; ++ci) {
        const int cp = lcls[M.off_loc + (long long)a * dpn + ci];
        any_row |= to_beta ? (cp == CLS_B || cp == CLS_C) : cp == CLS_I;
    }
    if (!any_row) return;
    const int ax = a % M.nn[0], ay = (a / M.nn[0]) % M.nn[1], az = a / (M.nn[0] * M.nn[1]);
    const int ex_max = M.nn[0] - 1, ey_max = M.nn[1] - 1, ez_max = dim == 3 ? M.nn[2] - 1 : 1;
    const int zlo = dim == 3 ? -1 : 0, zhi = dim == 3 ? 1 : 0;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int dz = zlo; dz <= zhi; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int bx = ax + dx, by = ay + dy, bz = az + dz;
                if (bx < 0 || by < 0 || bz < 0 || bx >= M.nn[0] || by >= M.nn[1] || bz >= M.nn[2]) continue;
                const int b = bx + M.nn[0] * (by + M.nn[1] * bz);
                // column DOFs of b in the input class, and their input values
                double xin[3] = {0.0, 0.0, 0.0};
                bool any_col = false;
                for (int cj = 0; cj < dpn; ++cj) {
                    const long long ql = M.off_loc + (long long)b * dpn + cj;
                    const int cq = lcls[ql], iq = lidx[ql];
                    if (to_beta ? cq == CLS_I : (cq == CLS_B || cq == CLS_C)) {
                        any_col = true;
                        xin[cj] = to_beta ? in[M.off_i + iq] : in[ob + (cq == CLS_B ? iq : M.n_b + iq)];
                    }
                }
                if (!any_col) continue;
                double blk[9];
                for (int q = 0; q < 9; ++q) blk[q] = 0.0;
                const int ex0 = max(max(ax, bx) - 1, 0), ex1 = min(min(ax, bx), ex_max - 1);
                const int ey0 = max(max(ay, by) - 1, 0), ey1 = min(min(ay, by), ey_max - 1);
                const int ez0 = dim == 3 ? max(max(az, bz) - 1, 0) : 0;
                const int ez1 = dim == 3 ? min(min(az, bz), ez_max - 1) : 0;
                for (int ez = ez0; ez <= ez1; ++ez)
                    for (int ey = ey0; ey <= ey1; ++ey)
                        for (int ex = ex0; ex <= ex1; ++ex) {
                            const int ca = (ax - ex) + 2 * (ay - ey) + (dim == 3 ? 4 * (az - ez) : 0);
                            const int cb = (bx - ex) + 2 * (by - ey) + (dim == 3 ? 4 * (bz - ez) : 0);
                            const long long ge = M.el0 + (long long)(M.lo[0] + ex) +
                                                 (long long)M.nelx * ((M.lo[1] + ey) + (long long)M.nely * (M.lo[2] + ez));
                            const double E = Emod[ge];
                            for (int ci = 0; ci < dpn; ++ci)
                                for (int cj = 0; cj < dpn; ++cj)
                                    blk[ci * dpn + cj] += E * K0[(ca * dpn + ci) * ne + cb * dpn + cj];
                        }
                // xin is zero for the DOFs of b outside the input class (fixed ones included)
                for (int ci = 0; ci < dpn; ++ci)
                    for (int cj = 0; cj < dpn; ++cj) acc[ci] = fma(blk[ci * dpn + cj], xin[cj], acc[ci]);
            }
    for (int ci = 0; ci < dpn; ++ci) {
        const long long pl = M.off_loc + (long long)a * dpn + ci;
        const int cp = lcls[pl], ip = lidx[pl];
        if (to_beta) {
            if (cp == CLS_B || cp == CLS_C) {
                const long long o = ob + (cp == CLS_B ? ip : M.n_b + ip);
                out[o] = f[o] - acc[ci];
            }
        } else if (cp == CLS_I) {
            out[M.off_i + ip] = f[M.off_i + ip] - acc[ci];
        }
    }
}

void launch_coupling(const DevTopo& t, const double* Emod, int to_beta, const double* in, const double* f, double* out,
                     hipStream_t st) {
    dim3 grid((t.max_nodes + 255) / 256, t.n_sub);
    k_coupling<<<grid, 256, 0, st>>>(t.subs, t.dim, t.K0dev, Emod, t.lcls, t.lidx, to_beta, in, f, out);
}

// SIMP moduli (Sec. 1, Eq. 1): E_e = Emin + rho_e^p (E0 - Emin), once per setup for the assembly
// and the coupling rows of the solve
__global__ void k_simp_moduli(long long n, const double* __restrict__ rho, double p, double E0, double Emin,
                              double* __restrict__ Emod) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e < n) Emod[e] = Emin + pow(rho[e], p) * (E0 - Emin);
}

void launch_simp_moduli(long long n, const double* rho, double p, double E0, double Emin, double* Emod,
                        hipStream_t st) {
    if (n > 0) k_simp_moduli<<<(int)((n + 255) / 256), 256, 0, st>>>(n, rho, p, E0, Emin, Emod);
}

// ---------------------------------------------------------------------------------------
// Block-tridiagonal Cholesky of K_ii, blocks = grid lines (2D) or planes (3D), for lines of more
// than 128 DOFs: plane by plane, each step batched over the subdomains,
//   D_k = A_kk - C_k C_k^T          (k_plane_syrk: one workgroup per 64 x 64 lower tile)
//   D_k = L_kk L_kk^T               (batched Cholesky, one workgroup per subdomain)
//   C_{k+1} = A_{k+1,k} L_kk^{-T}   (k_plane_trsm: one workgroup per 64 rows of C_{k+1})
// with C_k = L_{k,k-1} (row-major n_k x n_{k-1}, written over A_{k,k-1}).
__global__ void __launch_bounds__(256) k_plane_syrk(const SubMeta* __restrict__ subs,
                                                    const LineMeta* __restrict__ lines, int k, double* Lbuf) {
    __shared__ double lds[kLdsDoubles];
    const SubMeta M = subs[blockIdx.y];
    if (k >= M.n_lines) return;
    const LineMeta Lk = lines[M.line0 + k];
    const int nb = (Lk.n + 63) >> 6, t = blockIdx.x;
    if (Lk.n_prev == 0 || t >= nb * (nb + 1) / 2) return;
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = t - I * (I + 1) / 2;
    const double* Ls = Lbuf + Lk.off_sub;
    wg_gemm_sub(min(64, Lk.n - 64 * I), min(64, Lk.n - 64 * J), Lk.n_prev, Ls + 64ll * I * Lk.n_prev, Lk.n_prev, 1,
                Ls + 64ll * J * Lk.n_prev, 1, Lk.n_prev, Lbuf + Lk.off_diag + 64ll * I * Lk.n + 64 * J, Lk.n, 1,
                false, lds);
}

__global__ void __launch_bounds__(256) k_plane_trsm(const SubMeta* __restrict__ subs,
                                                    const LineMeta* __restrict__ lines, int k, double* Lbuf) {
    __shared__ double lds[kLdsDoubles];
    const SubMeta M = subs[blockIdx.y];
    if (k + 1 >= M.n_lines) return;
    const LineMeta Lk = lines[M.line0 + k], Ln = lines[M.line0 + k + 1];
    const int c0 = blockIdx.x * 64;
    if (Lk.n == 0 || c0 >= Ln.n) return;
    // rows c0 .. c0+63 of X = A_{k+1,k} L_kk^{-T}: solve L_kk X^T = A^T in place (X^T(i, c) = X[c][i])
    wg_trsm_lower(Lk.n, min(64, Ln.n - c0), Lbuf + Lk.off_diag, Lk.n, Lbuf + Ln.off_sub + (long long)c0 * Lk.n, 1,
                  Lk.n, lds);
}

// Cholesky descriptor of plane k of every subdomain (empty past its last plane), and the
// per-plane pivot flags cleared.
__global__ void k_plane_descs(const SubMeta* __restrict__ subs, int ns, const LineMeta* __restrict__ lines,
                              int np, PotrfDesc* __restrict__ pd, int* __restrict__ pinfo) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ns * np) return;
    const int k = e / ns;
    const SubMeta M = subs[e - k * ns];
    PotrfDesc d{0, 0, 1};
    if (k < M.n_lines) {
        const LineMeta L = lines[M.line0 + k];
        d = PotrfDesc{L.off_diag, L.n, max(L.n, 1)};
    }
    pd[e] = d;
    pinfo[e] = 0;
}

// info[s] = 0, or 1 + the interior DOF of the first non-positive pivot of subdomain s.
__global__ void k_plane_info(const SubMeta* __restrict__ subs, int ns, const LineMeta* __restrict__ lines, int np,
                             const int* __restrict__ pinfo, int* __restrict__ info) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const SubMeta M = subs[s];
    int v = 0;
    for (int k = 0; k < min(np, M.n_lines) && v == 0; ++k) {
        const int r = pinfo[(long long)k * ns + s];
        if (r) v = lines[M.line0 + k].i0 + r;
    }
    info[s] = v;
}

// Z <- L^{-1} Z for one chunk of 64 columns of Z = K_i,beta (row-major n_i x n_beta).
__global__ void __launch_bounds__(256) k_bt_forward(const SubMeta* __restrict__ subs,
                                                    const LineMeta* __restrict__ lines,
                                                    const double* __restrict__ Lbuf, double* Zbuf) {
    __shared__ double lds[kLdsDoubles];
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int c0 = blockIdx.x * 64;
    if (c0 >= M.n_beta || M.n_i == 0) return;
    const int nc = min(64, M.n_beta - c0);
    double* Z = Zbuf + M.off_Z + c0;
    for (int k = 0; k < M.n_lines; ++k) {
        const LineMeta Lk = lines[M.line0 + k];
        if (Lk.n == 0) continue;
        double* Zk = Z + (long long)Lk.i0 * M.n_beta;
        if (Lk.n_prev > 0) {
            const double* Zp = Z + (long long)(Lk.i0 - Lk.n_prev) * M.n_beta;
            wg_gemm_sub(Lk.n, nc, Lk.n_prev, Lbuf + Lk.off_sub, Lk.n_prev, 1, Zp, M.n_beta, 1, Zk, M.n_beta, 1,
                        false, lds);
        }
        wg_trsm_lower(Lk.n, nc, Lbuf + Lk.off_diag, Lk.n, Zk, M.n_beta, 1, lds);
    }
}

// Block-tridiagonal Cholesky of K_ii for lines of at most 128 DOFs, one workgroup per
// subdomain, the line's diagonal block resident in LDS (stride 129):
//   D_k -= C_k C_k^T           (FP64 matrix cores, lower 16x16 blocks; C_k = L_{k,k-1})
//   D_k  = L_kk L_kk^T          (16-column panels: panel rows in registers, trailing update on
//                                the matrix cores)
//   L_kk^{-1}                   (16x16 diagonal inverses, then the block columns on the matrix cores)
//   C_{k+1} = A_{k+1,k} L_kk^{-T}  (matrix cores, B operand from LDS, written over A_{k+1,k})
// L_kk goes to its slot of L and L_kk^{-1} to the inverse buffer.
constexpr int kBfLd = 129;
typedef double v4w __attribute__((ext_vector_type(4)));

// Z <- L^{-1} Z (Z = K_i,beta, row-major n_i x n_beta) plane by plane with the explicit inverses
// Li_k = L_kk^{-1}, each step batched over the subdomains on the FP64 matrix cores:
//   MODE 0:  T_k = Z_k - C_k Z_{k-1}     (T_k in a work buffer, one n_k x n_beta block per subdomain)
//   MODE 1:  Z_k = Li_k T_k              (Li_k lower triangular: columns past the row tile skipped)
// Workgroup: one 64 x 64 output tile (blockIdx.x = row tile + ntr * column tile), four wavefronts
// of 32 x 32; operands staged through LDS 16 deep. Lane (m, g) supplies A[row m][4s + g] and
// B[4s + g][column m] at sub-step s; its results are rows g + 4v, column m of each 16 x 16 block.
constexpr int kPfLd = 68;   // padded LDS row (doubles)
template <int MODE>
__global__ void __launch_bounds__(256) k_plane_fwd(const SubMeta* __restrict__ subs,
                                                   const LineMeta* __restrict__ lines, int k, int ntr,
                                                   const double* __restrict__ Lbuf, const double* __restrict__ Li,
                                                   double* Z, double* T, long long tstride) {
    __shared__ double As[16 * kPfLd], Bs[16 * kPfLd];
    const SubMeta M = subs[blockIdx.y];
    if (k >= M.n_lines) return;
    const LineMeta Lk = lines[M.line0 + k];
    const int r0 = 64 * (blockIdx.x % ntr), c0 = 64 * (blockIdx.x / ntr), nb = M.n_beta, n = Lk.n;
    if (r0 >= n || c0 >= nb) return;
    double* Zk = Z + M.off_Z + (long long)Lk.i0 * nb;
    double* Tk = T + tstride * blockIdx.y;
    const double* A;
    const double* B;
    int K, lda;
    if (MODE == 0) {
        A = Lbuf + Lk.off_sub;
        lda = Lk.n_prev;
        K = Lk.n_prev;
        B = Zk - (long long)Lk.n_prev * nb;
    } else {
        A = Li + Lk.off_inv;
        lda = n;
        K = min(n, r0 + 64);
        B = Tk;
    }
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
    const int wr = 32 * (wave & 1), wc = 32 * (wave >> 1);
    v4w acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4w{0.0, 0.0, 0.0, 0.0};
    for (int q0 = 0; q0 < K; q0 += 16) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int e = tid + 256 * p;
            const int qa = e & 15, ia = e >> 4;   // A: 16 consecutive columns of one row
            const int r = r0 + ia, qq = q0 + qa;
            As[qa * kPfLd + ia] = (r < n && qq < K) ? A[(long long)r * lda + qq] : 0.0;
            const int jb = e & 63, qb = e >> 6;   // B: 64 consecutive columns of one row
            const int qr = q0 + qb, cc = c0 + jb;
            Bs[qb * kPfLd + jb] = (qr < K && cc < nb) ? B[(long long)qr * nb + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int q = 4 * s4 + g;
            const double a0 = As[q * kPfLd + wr + m], a1 = As[q * kPfLd + wr + 16 + m];
            const double b0 = Bs[q * kPfLd + wc + m], b1 = Bs[q * kPfLd + wc + 16 + m];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = r0 + wr + 16 * i + g + 4 * v, col = c0 + wc + 16 * j + m;
                if (row < n && col < nb) {
                    const long long o = (long long)row * nb + col;
                    if (MODE == 0)
                        Tk[o] = Zk[o] - acc[i][j][v];
                    else
                        Zk[o] = acc[i][j][v];
                }
            }
}


// 32 operands of one 16-row block of a row-major matrix (rows r0 .. r0+15 of `rows`, columns
// 0 .. cols-1, zero outside) in the lane order of the 16x16x4 contractions: op[4Q + e] is row
// r0 + m, column 16Q + 4g + e. All loads are issued before any is used.
__device__ inline void bf_load_rowblock(double (&op)[32], const double* __restrict__ X, int r0, int rows, int cols) {
    const int lane = threadIdx.x & 63, m = lane & 15, g = lane >> 4, r = r0 + m;
#pragma unroll
    for (int Q = 0; Q < 8; ++Q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int q = 16 * Q + 4 * g + e;
            op[4 * Q + e] = (q < cols && r < rows) ? X[(long long)r * cols + q] : 0.0;
        }
}

__device__ inline void bf_syrk_update(double* A, const double* __restrict__ C, int n, int np) {
    // D -= C C^T on the lower 16x16 blocks of the n x n block (C is n x np). Wavefront w takes
    // block row w and, if it is 4 or more, block row nb-1-w (nb <= 8: every block row exactly once,
    // equal tile counts for nb = 8); the operands of a block row are loaded once, those of the next
    // tile while the current one is on the matrix cores.
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, m = lane & 15, g = lane >> 4;
    const int nb = (n + 15) >> 4;
    for (int pass = 0; pass < 2; ++pass) {
        const int bi = pass == 0 ? wave : nb - 1 - wave;
        if (bi >= nb || (pass == 1 && bi < 4)) continue;
        double a[32], b[32], bn[32];
        bf_load_rowblock(a, C, 16 * bi, n, np);
        bf_load_rowblock(b, C, 0, n, np);
        for (int bj = 0; bj <= bi; ++bj) {
            bf_load_rowblock(bn, C, 16 * (bj + 1), bj < bi ? n : 0, np);
            v4w acc = v4w{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int u = 0; u < 32; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
            // D layout: rows g + 4v, column m
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * bi + g + 4 * v, j = 16 * bj + m;
                if (i < n && j < n && j <= i) A[i * kBfLd + j] -= acc[v];
            }
#pragma unroll
            for (int u = 0; u < 32; ++u) b[u] = bn[u];
        }
    }
}

// Diagonal-block inverses of the line factor: 8 blocks of 16 x 16, row stride 17.
constexpr int kXdLd = 17;

// Blocked right-looking Cholesky of the lower triangle of A (n <= 128 DOFs, zero-padded to
// np = 16 ceil(n / 16) with every padded entry 0). Per 16-column panel: thread i (p0 <= i < np)
// keeps row i of the panel in registers and the 16 columns are eliminated in turn, the pivot column
// passing through LDS (double-buffered, one barrier a column); then the trailing lower triangle is
// updated, A_IK -= L_I,panel L_K,panel^T, in 16 x 16 tiles on the FP64 matrix cores. Afterwards the
// padded diagonal is set to 1, so L = diag(L_n, I). Returns 0 or the failing column + 1 (uniform).
__device__ inline int bf_potrf_blocked(double* A, int n, int np, double* colv /* 2 x 128 */) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
    const int nb = np >> 4;
    for (int p0 = 0; p0 < n; p0 += 16) {
        const int pb = min(16, n - p0), i = tid;
        const bool own = i >= p0 && i < np;
        double a[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) a[c] = (own && p0 + c <= i) ? A[i * kBfLd + p0 + c] : 0.0;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            double* cv = colv + 128 * (jj & 1);
            if (own) cv[i] = a[jj];
            __syncthreads();
            if (jj < pb) {
                const int j = p0 + jj;
                const double d = cv[j];
                if (!(d > 0.0)) return j + 1;
                const double piv = sqrt(d), inv = 1.0 / piv;
                const double li = (own && i > j) ? cv[i] * inv : 0.0;
                if (own && i >= j) a[jj] = i == j ? piv : li;
#pragma unroll
                for (int c = jj + 1; c < 16; ++c) a[c] = fma(-li, cv[p0 + c] * inv, a[c]);
            }
        }
        if (own) {
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (p0 + c <= i) A[i * kBfLd + p0 + c] = a[c];
        }
        __syncthreads();
        const int b1 = (p0 >> 4) + 1, mt = nb - b1, ntile = mt * (mt + 1) / 2;
        for (int t = wave; t < ntile; t += 4) {
            int I = 0;
            while ((I + 1) * (I + 2) / 2 <= t) ++I;
            const int K = t - I * (I + 1) / 2;
            const int r0 = 16 * (b1 + I), k0 = 16 * (b1 + K);
            v4w acc = v4w{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int q = p0 + g + 4 * kk;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(r0 + m) * kBfLd + q], A[(k0 + m) * kBfLd + q], acc, 0, 0, 0);
            }
            // D layout: rows g + 4v, column m
#pragma unroll
            for (int v = 0; v < 4; ++v) A[(r0 + g + 4 * v) * kBfLd + k0 + m] -= acc[v];
        }
        __syncthreads();
    }
    if (tid >= n && tid < np) A[tid * kBfLd + tid] = 1.0;
    __syncthreads();
    return 0;
}

// In-place inverse X = L^{-1} of the lower-triangular L in A (np x np, np a multiple of 16, unit
// padded diagonal). First the 16 x 16 diagonal blocks, X_II = L_II^{-1}, one thread per column by
// forward substitution into Xd; then block column J (wavefront J mod 4) from
//   X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ,   I = J+1, ...,
// on the FP64 matrix cores with the X_KJ tiles in registers (their accumulator layout is the
// operand layout of the next product). X_IJ goes to the unused upper block (J, I), transposed, and a
// last pass moves every block to its place in the lower triangle.
__device__ inline void bf_trtri_blocked(double* A, int np, double* Xd) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
    const int nb = np >> 4;
    if (tid < np) {
        const int I = tid >> 4, c = tid & 15;
        const double* L = A + 16 * I * kBfLd + 16 * I;
        double x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = r == c ? 1.0 : 0.0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            x[j] = x[j] / L[j * kBfLd + j];
#pragma unroll
            for (int r = j + 1; r < 16; ++r) x[r] = fma(-L[r * kBfLd + j], x[j], x[r]);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) Xd[(16 * I + r) * kXdLd + c] = x[r];
    }
    __syncthreads();
    for (int J = wave; J < nb; J += 4) {
        v4w xt[8];
#pragma unroll
        for (int K = 0; K < 8; ++K) {
#pragma unroll
            for (int v = 0; v < 4; ++v) xt[K][v] = K == J ? Xd[(16 * J + g + 4 * v) * kXdLd + m] : 0.0;
        }
#pragma unroll
        for (int I = 1; I < 8; ++I) {
            if (I > J && I < nb) {
                v4w t = v4w{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int K = 0; K < I; ++K) {
                    if (K >= J) {
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk)
                            t = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(16 * I + m) * kBfLd + 16 * K + g + 4 * kk],
                                                                     xt[K][kk], t, 0, 0, 0);
                    }
                }
                v4w x = v4w{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    x = __builtin_amdgcn_mfma_f64_16x16x4f64(Xd[(16 * I + m) * kXdLd + g + 4 * kk], t[kk], x, 0, 0, 0);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    xt[I][v] = -x[v];
                    A[(16 * J + m) * kBfLd + 16 * I + g + 4 * v] = -x[v];
                }
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < np * np; e += 256) {
        const int i = e / np, c = e - i * np;
        if (c > i) continue;
        A[i * kBfLd + c] = (i >> 4) == (c >> 4) ? Xd[i * kXdLd + (c & 15)] : A[c * kBfLd + i];
    }
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_bt_factor128(const SubMeta* __restrict__ subs, const LineMeta* __restrict__ lines,
                                                      double* Lbuf, double* Li, int* info) {
    __shared__ double A[128 * kBfLd];
    __shared__ double colv[256];
    __shared__ double Xd[128 * kXdLd];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
    for (int k = 0; k < M.n_lines; ++k) {
        const LineMeta Lk = lines[M.line0 + k];
        const int n = Lk.n;
        if (n == 0) continue;
        const int np = (n + 15) & ~15;
        double* D = Lbuf + Lk.off_diag;
        for (int e0 = tid; e0 < np * np; e0 += 8 * 256) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + 256 * u, i = e / np, j = e - i * np;
                v[u] = (e < np * np && i < n && j < n) ? D[i * n + j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + 256 * u, i = e / np, j = e - i * np;
                if (e < np * np) A[i * kBfLd + j] = v[u];
            }
        }
        __syncthreads();
        if (Lk.n_prev > 0) {
            bf_syrk_update(A, Lbuf + Lk.off_sub, n, Lk.n_prev);
            __syncthreads();
        }
        const int r = bf_potrf_blocked(A, n, np, colv);
        if (r) {
            if (tid == 0) info[s] = Lk.i0 + r;
            return;
        }
        for (int e = tid; e < n * n; e += 256) {
            const int i = e / n, j = e - i * n;
            D[e] = j <= i ? A[i * kBfLd + j] : 0.0;
        }
        __syncthreads();
        bf_trtri_blocked(A, np, Xd);
        double* X = Li + Lk.off_inv;
        for (int e = tid; e < n * n; e += 256) {
            const int i = e / n, j = e - i * n;
            X[e] = j <= i ? A[i * kBfLd + j] : 0.0;
        }
        if (k + 1 < M.n_lines) {
            const LineMeta Ln = lines[M.line0 + k + 1];
            if (Ln.n > 0) {
                // C = A_{k+1,k} L_kk^{-T}: C[r][c] = sum_{q <= c} A[r][q] X[c][q]; wavefront = 16 rows
                // x all columns, every row block read completely before it is overwritten
                double* Ab = Lbuf + Ln.off_sub;   // n_next x n
                const int nn = Ln.n, ncb = (n + 15) >> 4;
                double a[32];
                if (wave < (nn + 15) / 16) bf_load_rowblock(a, Ab, 16 * wave, nn, n);
                for (int rbk = wave; rbk < (nn + 15) / 16; rbk += 4) {
                    double an[32];
                    bf_load_rowblock(an, Ab, 16 * (rbk + 4), rbk + 4 < (nn + 15) / 16 ? nn : 0, n);
                    v4w acc[8];
#pragma unroll
                    for (int cb = 0; cb < 8; ++cb) acc[cb] = v4w{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int u = 0; u < 32; ++u) {
                        const int q = 16 * (u >> 2) + 4 * g + (u & 3);
#pragma unroll
                        for (int cb = 0; cb < 8; ++cb) {
                            if (cb < ncb) {
                                const int cc = 16 * cb + m;
                                const double b = (q < n && cc < n && q <= cc) ? A[cc * kBfLd + q] : 0.0;
                                acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b, acc[cb], 0, 0, 0);
                            }
                        }
                    }
#pragma unroll
                    for (int cb = 0; cb < 8; ++cb)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int rr = 16 * rbk + g + 4 * v, cc = 16 * cb + m;
                            if (cb < ncb && rr < nn && cc < n) Ab[(long long)rr * n + cc] = acc[cb][v];
                        }
#pragma unroll
                    for (int u = 0; u < 32; ++u) a[u] = an[u];
                }
            }
        }
        __syncthreads();
    }
}

// Z <- L^{-1} Z for one 64-column chunk of Z = K_i,beta (row-major n_i x n_beta), with the
// explicit inverses L_kk^{-1} (lines of at most 128 DOFs): per line T = Z_k - L_{k,k-1} Z_{k-1},
// then Z_k = L_kk^{-1} T, both on the FP64 matrix cores. Z_{k-1} and then T stay in one LDS
// buffer (128 x 68); wavefront w computes rows 32w..32w+31 of the line (two 16-row blocks x
// four 16-column blocks). The contraction of step Q uses index 16Q + 4g + s for lane group g
// and sub-step s, so a lane's four operands of A are consecutive.
constexpr int kFwLd = 68;

__global__ void __launch_bounds__(256, 2) k_bt_forward_mfma(const SubMeta* __restrict__ subs,
                                                            const LineMeta* __restrict__ lines,
                                                            const double* __restrict__ Lbuf,
                                                            const double* __restrict__ Li, double* Zbuf) {
    __shared__ double buf[128 * kFwLd];
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int c0 = blockIdx.x * 64;
    if (c0 >= M.n_beta || M.n_i == 0) return;
    const int nc = min(64, M.n_beta - c0);
    double* Z = Zbuf + M.off_Z + c0;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
    const int rw = 32 * wave;   // first row of the wavefront within the line
    int n_prev = 0;
    for (int k = 0; k < M.n_lines; ++k) {
        const LineMeta Lk = lines[M.line0 + k];
        if (Lk.n == 0) {
            n_prev = 0;
            continue;
        }
        const int n = Lk.n, np = Lk.n_prev;
        double* Zk = Z + (long long)Lk.i0 * M.n_beta;
        v4w acc[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = v4w{0.0, 0.0, 0.0, 0.0};
        // acc = L_{k,k-1} Z_{k-1} (Z_{k-1} in buf, rows < np)
        if (np > 0 && n_prev == np && rw < n) {
            const double* C = Lbuf + Lk.off_sub;
            for (int Q = 0; Q < (np + 15) / 16; ++Q) {
                const int q0 = 16 * Q + 4 * g;
                double a0[4], a1[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int q = q0 + e;
                    const int r0 = rw + m, r1 = rw + 16 + m;
                    a0[e] = (q < np && r0 < n) ? C[(long long)r0 * np + q] : 0.0;
                    a1[e] = (q < np && r1 < n) ? C[(long long)r1 * np + q] : 0.0;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int q = q0 + e;
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb) {
                        const double bv = q < np ? buf[q * kFwLd + 16 * cb + m] : 0.0;
                        acc[0][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[e], bv, acc[0][cb], 0, 0, 0);
                        acc[1][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[e], bv, acc[1][cb], 0, 0, 0);
                    }
                }
            }
        }
        // T = Z_k - acc (D layout: rows g + 4v, column m of each block)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = rw + 16 * a + g + 4 * v, c = 16 * cb + m;
                    const double zk = (r < n && c < nc) ? Zk[(long long)r * M.n_beta + c] : 0.0;
                    acc[a][cb][v] = zk - acc[a][cb][v];
                }
        __syncthreads();   // every wavefront is done with Z_{k-1}
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v) buf[(rw + 16 * a + g + 4 * v) * kFwLd + 16 * cb + m] = acc[a][cb][v];
        __syncthreads();
        // Z_k = L_kk^{-1} T (lower triangular: contraction index q <= row)
        v4w z[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) z[a][b] = v4w{0.0, 0.0, 0.0, 0.0};
        if (rw < n) {
            const double* I = Li + Lk.off_inv;
            const int qmax = min(n, rw + 32);
            for (int Q = 0; Q < (qmax + 15) / 16; ++Q) {
                const int q0 = 16 * Q + 4 * g;
                double a0[4], a1[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int q = q0 + e;
                    const int r0 = rw + m, r1 = rw + 16 + m;
                    a0[e] = (q < n && r0 < n) ? I[(long long)r0 * n + q] : 0.0;
                    a1[e] = (q < n && r1 < n) ? I[(long long)r1 * n + q] : 0.0;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int q = q0 + e;
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb) {
                        const double bv = q < n ? buf[q * kFwLd + 16 * cb + m] : 0.0;
                        z[0][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[e], bv, z[0][cb], 0, 0, 0);
                        z[1][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[e], bv, z[1][cb], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();   // every wavefront is done with T
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = rw + 16 * a + g + 4 * v, c = 16 * cb + m;
                    buf[r * kFwLd + c] = z[a][cb][v];
                    if (r < n && c < nc) Zk[(long long)r * M.n_beta + c] = z[a][cb][v];
                }
        __syncthreads();
        n_prev = n;
    }
}

// ---------------------------------------------------------------------------------------
// Batched C = beta C + alpha A^T B (A: k x m, B: k x n, row-major with leading dimensions
// lda/ldb) on the FP64 matrix cores. Workgroup = one 64x64 tile of C; its four wavefronts
// split the contraction and each accumulates the full tile (sixteen 16x16 accumulators, one
// wavefront per SIMD, loads kGtRing steps ahead); the partial tiles meet in LDS and are summed
// in wavefront order. Rows and columns of the tile are permuted so that at step st lane
// (m, g) reads A[4 st + g][i0 + 4m .. +3] and B[4 st + g][j0 + 4m .. +3]: accumulator row m'
// of block ib is tile row 4 m' + ib, column n' of block jb is tile column 4 n' + jb.
// symmetric (A == B): only tiles on or below the diagonal are enumerated (tile t of a matrix is
// the t-th of the lower triangle, row by row); off-diagonal tiles are written to both (i, j) and
// (j, i). Placement: workgroups go to the eight XCDs in turn, so workgroup L serves matrix
// (L mod 8) + 8 ((L / 8) / tiles) and all tiles of one matrix run on one XCD, where the column
// blocks they share are read through one L2.
typedef double v4g __attribute__((ext_vector_type(4)));
constexpr int kGtRing = 6;

__global__ void __launch_bounds__(256, 1) k_gemm_tn(const GemmDesc* __restrict__ desc, int nbatch, const double* Abase,
                                                    const double* Bbase, double* Cbase, double alpha, double beta,
                                                    int symmetric) {
    __shared__ double red[4 * 4096];
    const int wl = blockIdx.x + gridDim.x * blockIdx.y, slot = wl >> 3;
    const int mat = (wl & 7) + 8 * (slot / (int)gridDim.x), tile = slot % (int)gridDim.x;
    if (mat >= nbatch) return;
    const GemmDesc d = desc[mat];
    int ti, tj;
    if (symmetric) {
        ti = 0;
        while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
        tj = tile - ti * (ti + 1) / 2;
    } else {
        const int tn = (d.n + 63) / 64;
        ti = tile / tn;
        tj = tile % tn;
    }
    if (ti * 64 >= d.m || tj * 64 >= d.n) return;
    const double* A = Abase + d.a;
    const double* B = Bbase + d.b;
    double* C = Cbase + d.c;
    const int i0 = ti * 64, j0 = tj * 64;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
    const int nsteps = (d.k + 3) >> 2;
    const int w0 = nsteps * wave / 4, w1 = nsteps * (wave + 1) / 4;
    const int ia = i0 + 4 * m, jb0 = j0 + 4 * m;
    v4g acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4g{0.0, 0.0, 0.0, 0.0};
    v4g ar[kGtRing], br[kGtRing];
    auto ld = [&](int st, v4g& av, v4g& bv) {
        const int r = 4 * st + g;
        const bool rv = st < w1 && r < d.k;
        const double* Ar = A + (long long)r * d.lda;
        const double* Br = B + (long long)r * d.ldb;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            av[e] = (rv && ia + e < d.m) ? Ar[ia + e] : 0.0;
            bv[e] = (rv && jb0 + e < d.n) ? Br[jb0 + e] : 0.0;
        }
    };
#pragma unroll
    for (int dd = 0; dd < kGtRing; ++dd) ld(w0 + dd, ar[dd], br[dd]);
    for (int st = w0; st < w1; st += kGtRing) {
#pragma unroll
        for (int dd = 0; dd < kGtRing; ++dd) {
            if (st + dd < w1) {
#pragma unroll
                for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                    for (int jb = 0; jb < 4; ++jb)
                        acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[dd][ib], br[dd][jb], acc[ib][jb], 0, 0, 0);
                ld(st + dd + kGtRing, ar[dd], br[dd]);
            }
        }
    }
    // D layout: lane holds rows g + 4v, column m of block (ib, jb) -> tile (4(g+4v)+ib, 4m+jb)
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[wave * 4096 + (4 * (g + 4 * v) + ib) * 64 + 4 * m + jb] = acc[ib][jb][v];
    __syncthreads();
    for (int e = tid; e < 4096; e += 256) {
        const int i = i0 + (e >> 6), j = j0 + (e & 63);
        if (i >= d.m || j >= d.n) continue;
        const double val = ((red[e] + red[4096 + e]) + red[8192 + e]) + red[12288 + e];
        double* dst = C + (long long)i * d.ldc + j;
        *dst = beta == 0.0 ? alpha * val : beta * *dst + alpha * val;
        if (symmetric && ti != tj) {
            double* dt = C + (long long)j * d.ldc + i;
            *dt = beta == 0.0 ? alpha * val : beta * *dt + alpha * val;
        }
    }
}

// Batched in-place Cholesky of matrices of at most 512 rows, one 512-thread workgroup per matrix,
// right-looking in 32-column panels. Thread i keeps row i of the panel in registers; the 32
// columns are eliminated in turn with the pivot column passing through LDS (double-buffered, one
// barrier a column). The finished panel goes to A and to LDS, and the trailing lower triangle is
// updated, A_IK -= L_I,panel L_K,panel^T, in 16x16 tiles on the FP64 matrix cores (operands from
// LDS, four tiles per wavefront in flight). Entries above the diagonal are left unspecified;
// info = 0 or the failing column + 1.
constexpr int kPpLd = 33;

__global__ void __launch_bounds__(512) k_potrf512(const PotrfDesc* __restrict__ desc, double* base, int* info) {
    __shared__ double P[512 * kPpLd];
    __shared__ double colv[2 * 512];
    const PotrfDesc d = desc[blockIdx.x];
    double* A = base + d.a;
    const long long lda = d.lda;
    const int n = d.n;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, m = lane & 15, g = lane >> 4;
    for (int k0 = 0; k0 < n; k0 += 32) {
        const int kb = min(32, n - k0), i = tid;
        const bool own = i >= k0 && i < n;
        double a[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) a[c] = (own && c < kb && k0 + c <= i) ? A[i * lda + k0 + c] : 0.0;
#pragma unroll
        for (int jj = 0; jj < 32; ++jj) {
            double* cv = colv + 512 * (jj & 1);
            if (own) cv[i] = a[jj];
            __syncthreads();
            if (jj < kb) {
                const int j = k0 + jj;
                const double dj = cv[j];
                if (!(dj > 0.0)) {   // uniform: every thread read the same value
                    if (tid == 0) info[blockIdx.x] = j + 1;
                    return;
                }
                const double piv = sqrt(dj), inv = 1.0 / piv;
                const double li = (own && i > j) ? cv[i] * inv : 0.0;
                if (own && i >= j) a[jj] = i == j ? piv : li;
#pragma unroll
                for (int c = jj + 1; c < 32; ++c) {
                    const double lk = k0 + c < n ? cv[k0 + c] * inv : 0.0;
                    a[c] = fma(-li, lk, a[c]);
                }
            }
        }
        if (own) {
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                if (c < kb && k0 + c <= i) A[i * lda + k0 + c] = a[c];
                P[i * kPpLd + c] = a[c];
            }
        }
        __syncthreads();
        const int t0 = k0 + kb, nbt = (n - t0 + 15) >> 4, ntile = nbt * (nbt + 1) / 2;
        for (int tb = 4 * wave; tb < ntile; tb += 32) {
            int r0[4], c0[4];
            double cval[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = min(tb + u, ntile - 1);
                int I = 0;
                while ((I + 1) * (I + 2) / 2 <= t) ++I;
                r0[u] = t0 + 16 * I;
                c0[u] = t0 + 16 * (t - I * (I + 1) / 2);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0[u] + g + 4 * v, c = c0[u] + m;
                    cval[u][v] = (tb + u < ntile && r < n && c < n) ? A[r * lda + c] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v4g acc = v4g{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 8; ++kk)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(P[(r0[u] + m) * kPpLd + 4 * kk + g],
                                                               P[(c0[u] + m) * kPpLd + 4 * kk + g], acc, 0, 0, 0);
                // D layout: rows g + 4v, column m
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0[u] + g + 4 * v, c = c0[u] + m;
                    if (tb + u < ntile && r < n && c < n) A[r * lda + c] = cval[u][v] - acc[v];
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) info[blockIdx.x] = 0;
}

// Blocked batched Cholesky for large matrices, three launches per panel of kPfB columns
// starting at p0 (every matrix of the batch advances in step; matrices already finished, or
// with a failed pivot, skip):
//   k_potrf_diag:  A11 = L11 L11^T in place, one workgroup per matrix;
//   k_potrf_panel: L21 = A21 L11^{-T}, kPfRows rows per workgroup (one thread per row,
//                  substitution against L11 in LDS);
//   k_potrf_syrk:  A22 -= L21 L21^T on the lower 64x64 tiles of the trailing matrix, one
//                  workgroup per tile (FP64 matrix cores, operands in LDS).
// info[b]: 0, or 1 + the column of the first non-positive pivot (as the one-workgroup form).
constexpr int kPfB = 64, kPfRows = 128;
__global__ void __launch_bounds__(256) k_potrf_diag(const PotrfDesc* __restrict__ desc, int p0, double* base,
                                                    int* info) {
    __shared__ double lds[kLdsDoubles];
    const PotrfDesc d = desc[blockIdx.x];
    if (p0 >= d.n || (p0 > 0 && info[blockIdx.x] != 0)) return;   // uniform
    const int b = min(kPfB, d.n - p0);
    const int r = wg_potrf(b, base + d.a + (long long)p0 * d.lda + p0, d.lda, lds);
    if (threadIdx.x == 0 && (r || p0 == 0)) info[blockIdx.x] = r ? p0 + r : 0;
}

__global__ void __launch_bounds__(256) k_potrf_panel(const PotrfDesc* __restrict__ desc, int p0, double* base,
                                                     const int* __restrict__ info) {
    __shared__ double Ls[kPfB][kPfB + 1];
    __shared__ double Xs[kPfRows][kPfB + 1];
    const PotrfDesc d = desc[blockIdx.y];
    if (p0 >= d.n) return;
    const int b = min(kPfB, d.n - p0);
    const int r0 = p0 + b + blockIdx.x * kPfRows;
    if (r0 >= d.n || info[blockIdx.y] != 0) return;   // uniform
    const int nr = min(kPfRows, d.n - r0);
    double* A = base + d.a;
    for (int e = threadIdx.x; e < kPfB * kPfB; e += 256) {
        const int i = e / kPfB, j = e % kPfB;
        Ls[i][j] = (i < b && j <= i) ? A[(long long)(p0 + i) * d.lda + p0 + j] : 0.0;
    }
    for (int e = threadIdx.x; e < kPfRows * kPfB; e += 256) {
        const int i = e / kPfB, j = e % kPfB;
        Xs[i][j] = (i < nr && j < b) ? A[(long long)(r0 + i) * d.lda + p0 + j] : 0.0;
    }
    __syncthreads();
    if ((int)threadIdx.x < nr) {
        const int i = threadIdx.x;
        for (int j = 0; j < b; ++j) {
            double v = Xs[i][j];
            for (int k = 0; k < j; ++k) v -= Xs[i][k] * Ls[j][k];
            Xs[i][j] = v / Ls[j][j];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kPfRows * kPfB; e += 256) {
        const int i = e / kPfB, j = e % kPfB;
        if (i < nr && j < b) A[(long long)(r0 + i) * d.lda + p0 + j] = Xs[i][j];
    }
}

// Trailing update with the factored panel columns p0 .. q0-1 (q0 = p0 + min(kw, n - p0), kw = 64
// or 128, staged 64 at a time): strip = 0 updates every lower 64 x 64 tile of the trailing matrix
// (rows and columns >= q0), strip = 1 only the tiles of its first 64 columns (the next panel).
__global__ void __launch_bounds__(256) k_potrf_syrk(const PotrfDesc* __restrict__ desc, int p0, int kw, int strip,
                                                    double* base, const int* __restrict__ info) {
    __shared__ double Ai[64][kPfB + 1];
    __shared__ double Aj[64][kPfB + 1];
    const PotrfDesc d = desc[blockIdx.y];
    if (p0 >= d.n) return;
    const int kcols = min(kw, d.n - p0), q0 = p0 + kcols;
    const int nt = (d.n - q0 + 63) / 64;
    const int t = blockIdx.x;
    int I = t, J = 0;
    if (!strip) {
        I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        while (I * (I + 1) / 2 > t) --I;
        J = t - I * (I + 1) / 2;
    }
    if (I >= nt || info[blockIdx.y] != 0) return;   // uniform
    double* A = base + d.a;
    const int ri = q0 + 64 * I, rj = q0 + 64 * J;
    // FP64 matrix cores: wavefront w takes the 32 x 32 quadrant (rows 32 (w & 1), columns
    // 32 (w >> 1)); lane (m, g) supplies Ai[row m][4s + g] and Aj[column m][4s + g] at sub-step s,
    // and holds rows g + 4v, column m of each 16 x 16 block. The quadrant above the diagonal of a
    // diagonal tile only stages.
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, m = lane & 15, g = lane >> 4;
    const int wr = 32 * (wave & 1), wc = 32 * (wave >> 1);
    const bool work = !(J == I && wc > wr);
    v4w acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = v4w{0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < kcols; kc += kPfB) {
        if (kc) __syncthreads();
        for (int e = threadIdx.x; e < 64 * kPfB; e += 256) {
            const int i = e / kPfB, k = e % kPfB;
            const bool kin = kc + k < kcols;
            Ai[i][k] = (ri + i < d.n && kin) ? A[(long long)(ri + i) * d.lda + p0 + kc + k] : 0.0;
            Aj[i][k] = (rj + i < d.n && kin) ? A[(long long)(rj + i) * d.lda + p0 + kc + k] : 0.0;
        }
        __syncthreads();
        if (work) {
#pragma unroll 4
            for (int k = 0; k < kPfB; k += 4) {
                const double a0 = Ai[wr + m][k + g], a1 = Ai[wr + 16 + m][k + g];
                const double b0 = Aj[wc + m][k + g], b1 = Aj[wc + 16 + m][k + g];
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
            }
        }
    }
    if (!work) return;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = ri + wr + 16 * x + g + 4 * v, j = rj + wc + 16 * y + m;
                if (i < d.n && j <= i) A[(long long)i * d.lda + j] -= acc[x][y][v];
            }
}

// Batched B <- L^{-1} B for B holding the identity on entry (the explicit inverse of a
// Cholesky factor), one workgroup per (matrix, chunk of 64 columns of B). Rows above the chunk's
// first column are zero in B and stay zero in L^{-1} B (L lower triangular), so the chunk's
// substitution starts at that row, on the trailing block of L.
__global__ void __launch_bounds__(256) k_trsm(const TrsmDesc* __restrict__ desc, const double* Lbase,
                                              double* Bbase) {
    __shared__ double lds[kLdsTrsm64];
    const TrsmDesc d = desc[blockIdx.y];
    const int c0 = blockIdx.x * 64;
    if (c0 >= d.ncols || c0 >= d.n) return;
    const int nc = min(64, d.ncols - c0);
    wg_trsm_lower<64>(d.n - c0, nc, Lbase + d.l + (long long)c0 * d.ldl + c0, d.ldl, Bbase + d.b + (long long)c0 * d.ldb + c0,
                  d.ldb, 1, lds);
}

// ---------------------------------------------------------------------------------------
// Element-wise helpers on per-subdomain square blocks.

// dst[s] (n_b x n_b, ld n_b) = S_bb of subdomain s (the leading block of S, ld n_beta);
// identity != 0 writes the identity instead.
__global__ void k_copy_Sbb(const SubMeta* __restrict__ subs, const double* __restrict__ Sbuf, double* dst,
                           int identity) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const long long nn = (long long)M.n_b * M.n_b;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / M.n_b), j = (int)(e % M.n_b);
        dst[M.off_P + e] = identity ? (i == j ? 1.0 : 0.0) : Sbuf[M.off_S + (long long)i * M.n_beta + j];
    }
}

// Pk[s]: the leading n_b x n_b block of S (ld n_beta) as its upper triangle in 64x64 tiles, tile
// (I, J), I <= J, at (J(J+1)/2 + I) * 4096 with element (a, b) = S[64I + a][64J + b], zero past n_b
__global__ void k_pack_sym(const SubMeta* __restrict__ subs, const double* __restrict__ Sbuf, double* __restrict__ Pk) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int nT = (M.n_b + 63) >> 6;
    const long long ne = (long long)nT * (nT + 1) / 2 * 4096;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne; e += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(e >> 12), a = (int)((e >> 6) & 63), b = (int)(e & 63);
        int J = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
        while ((J + 1) * (J + 2) / 2 <= t) ++J;
        while (J * (J + 1) / 2 > t) --J;
        const int I = t - J * (J + 1) / 2;
        const int row = 64 * I + a, col = 64 * J + b;
        Pk[M.off_Pk + e] = (row < M.n_b && col < M.n_b) ? Sbuf[M.off_S + (long long)row * M.n_beta + col] : 0.0;
    }
}

// ---------------------------------------------------------------------------------------
// TFETI: rigid-body modes restricted to the interface DOFs b, orthonormalised
// (Rhat_b = R_b C^{-T}, C C^T = R_b^T R_b), and the regularised matrix
// W = S_bb + tau Rhat Rhat^T whose inverse gives the pseudo-inverse
// S_bb^+ = W^{-1} - Rhat Rhat^T / tau (exact when S_bb R_b = 0).
__device__ inline void rbm_row(int dim, int comp, double x, double y, double z, double* r) {
    // translations, then rotations about z, x, y: (-y, x, 0), (0, -z, y), (z, 0, -x)
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

__device__ inline void local_dof_coords(const SubMeta& M, int dim, int l, int* comp, double* x, double* y,
                                        double* z) {
    const int node = l / dim;
    *comp = l % dim;
    const int ix = node % M.nn[0], iy = (node / M.nn[0]) % M.nn[1], iz = node / (M.nn[0] * M.nn[1]);
    *x = ix - 0.5 * (M.nn[0] - 1);
    *y = iy - 0.5 * (M.nn[1] - 1);
    *z = iz - 0.5 * (M.nn[2] - 1);
}

__global__ void __launch_bounds__(256) k_tfeti_rbm(const SubMeta* __restrict__ subs, int dim,
                                                   const int* __restrict__ b_loc, const double* __restrict__ Sbuf,
                                                   double* Rb, double* Cit, double* tau, double* Wbuf) {
    __shared__ double red[256][21];
    __shared__ double Gm[36], Ci[36];
    __shared__ double tsum[256];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    const int nm = dim == 2 ? 3 : 6;
    const int tid = threadIdx.x;
    double g[21];
    for (int q = 0; q < 21; ++q) g[q] = 0.0;
    double dsum = 0.0;
    for (int j = tid; j < M.n_b; j += 256) {
        int comp;
        double x, y, z, r[6];
        local_dof_coords(M, dim, b_loc[M.off_b + j], &comp, &x, &y, &z);
        rbm_row(dim, comp, x, y, z, r);
        int q = 0;
        for (int a = 0; a < nm; ++a)
            for (int b = 0; b <= a; ++b) g[q++] += r[a] * r[b];
        dsum += Sbuf[M.off_S + (long long)j * M.n_beta + j];
    }
    for (int q = 0; q < 21; ++q) red[tid][q] = g[q];
    tsum[tid] = dsum;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int u = 0; u < 256; ++u) t += tsum[u];
        tau[s] = t / M.n_b;
        int q = 0;
        for (int a = 0; a < nm; ++a)
            for (int b = 0; b <= a; ++b) {
                double v = 0.0;
                for (int u = 0; u < 256; ++u) v += red[u][q];
                Gm[a * nm + b] = v;
                Gm[b * nm + a] = v;
                ++q;
            }
        // Cholesky Gm = C C^T (lower), then Ci = C^{-T} (upper)
        double C[36];
        for (int a = 0; a < nm; ++a)
            for (int b = 0; b < nm; ++b) C[a * nm + b] = 0.0;
        for (int j = 0; j < nm; ++j) {
            double d = Gm[j * nm + j];
            for (int k = 0; k < j; ++k) d -= C[j * nm + k] * C[j * nm + k];
            d = sqrt(d);
            C[j * nm + j] = d;
            for (int i = j + 1; i < nm; ++i) {
                double v = Gm[i * nm + j];
                for (int k = 0; k < j; ++k) v -= C[i * nm + k] * C[j * nm + k];
                C[i * nm + j] = v / d;
            }
        }
        // inverse of lower C, then transpose
        double Inv[36];
        for (int c = 0; c < nm; ++c)
            for (int i = 0; i < nm; ++i) {
                double v = i == c ? 1.0 : 0.0;
                for (int k = 0; k < i; ++k) v -= C[i * nm + k] * Inv[k * nm + c];
                Inv[i * nm + c] = v / C[i * nm + i];
            }
        for (int a = 0; a < nm; ++a)
            for (int b = 0; b < nm; ++b) {
                Ci[a * nm + b] = Inv[b * nm + a];
                Cit[s * 36 + a * nm + b] = Inv[b * nm + a];
            }
    }
    __syncthreads();
    for (int j = tid; j < M.n_b; j += 256) {
        int comp;
        double x, y, z, r[6];
        local_dof_coords(M, dim, b_loc[M.off_b + j], &comp, &x, &y, &z);
        rbm_row(dim, comp, x, y, z, r);
        for (int m = 0; m < nm; ++m) {
            double v = 0.0;
            for (int a = 0; a < nm; ++a) v += r[a] * Ci[a * nm + m];
            Rb[M.off_R + (long long)j * nm + m] = v;
        }
    }
    __syncthreads();
    const double t = tau[s];
    const long long nn = (long long)M.n_b * M.n_b;
    for (long long e = tid; e < nn; e += 256) {
        const int i = (int)(e / M.n_b), j = (int)(e % M.n_b);
        double v = 0.0;
        for (int m = 0; m < nm; ++m) v += Rb[M.off_R + (long long)i * nm + m] * Rb[M.off_R + (long long)j * nm + m];
        Wbuf[M.off_P + e] = Sbuf[M.off_S + (long long)i * M.n_beta + j] + t * v;
    }
}

// F_s -= Rhat Rhat^T / tau (TFETI pseudo-inverse correction).
__global__ void k_tfeti_fix(const SubMeta* __restrict__ subs, int nm, const double* __restrict__ Rb,
                            const double* __restrict__ tau, double* F64) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const long long nn = (long long)M.n_b * M.n_b;
    const double it = 1.0 / tau[s];
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / M.n_b), j = (int)(e % M.n_b);
        double v = 0.0;
        for (int m = 0; m < nm; ++m) v += Rb[M.off_R + (long long)i * nm + m] * Rb[M.off_R + (long long)j * nm + m];
        F64[M.off_F + (long long)i * M.ldF + j] -= it * v;
    }
}

// FETI-DP: F_rc^T = S_cb F_s (rows n_b.. of the augmented operator) and
// Kbar_cc^s = S_cc - S_cb F_s S_bc (eliminating b after i from the interface Schur complement).
// Pass 1: workgroup (x, s) takes columns j = 256 x + t of F_s; a thread keeps the n_c (<= 32)
// outputs of its column in registers and streams its column of F_s once (coalesced over the
// workgroup), with S_cb staged through LDS in slices of kFrcSlice columns (zero rows past n_c).
constexpr int kFrcSlice = 64;
__global__ void __launch_bounds__(256) k_frc(const SubMeta* __restrict__ subs, const double* __restrict__ Sbuf,
                                             double* F64) {
    __shared__ __attribute__((aligned(16))) double Sc[kFrcSlice][32];   // Sc[q][c] = S_cb[c][q0 + q]
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const int nb = M.n_b, nc = M.n_c;
    if (nc == 0 || blockIdx.x * 256 >= nb) return;   // uniform over the workgroup
    const int j = blockIdx.x * 256 + threadIdx.x;
    const double* S = Sbuf + M.off_S;
    double* F = F64 + M.off_F;
    double v[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) v[c] = 0.0;
    for (int q0 = 0; q0 < nb; q0 += kFrcSlice) {
        const int qn = min(kFrcSlice, nb - q0);
        __syncthreads();   // the previous slice is consumed
        for (int e = threadIdx.x; e < kFrcSlice * 32; e += 256) {
            const int q = e % kFrcSlice, c = e / kFrcSlice;
            Sc[q][c] = (q < qn && c < nc) ? S[(long long)(nb + c) * M.n_beta + q0 + q] : 0.0;
        }
        __syncthreads();
        if (j < nb) {
#pragma unroll 4
            for (int q = 0; q < qn; ++q) {
                const double f = F[(long long)(q0 + q) * M.ldF + j];
#pragma unroll
                for (int c = 0; c < 32; c += 2) {
                    const double2 sc = *reinterpret_cast<const double2*>(&Sc[q][c]);
                    v[c] = fma(sc.x, f, v[c]);
                    v[c + 1] = fma(sc.y, f, v[c + 1]);
                }
            }
        }
    }
    if (j < nb)
#pragma unroll
        for (int c = 0; c < 32; ++c)
            if (c < nc) F[(long long)(M.rowT + c) * M.ldF + j] = v[c];
}

// Pass 2: Kbar_cc^s = S_cc - F_rc^T S_bc, one workgroup per subdomain, one thread per entry.
__global__ void __launch_bounds__(256) k_frc_kc(const SubMeta* __restrict__ subs, const double* __restrict__ Sbuf,
                                                const double* __restrict__ F64, double* Kc) {
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    const int nb = M.n_b, nc = M.n_c;
    const double* S = Sbuf + M.off_S;
    const double* F = F64 + M.off_F;
    for (int e = threadIdx.x; e < nc * nc; e += 256) {
        const int c = e / nc, c2 = e % nc;
        double v = S[(long long)(nb + c) * M.n_beta + nb + c2];
        for (int j = 0; j < nb; ++j) v -= F[(long long)(M.rowT + c) * M.ldF + j] * S[(long long)j * M.n_beta + nb + c2];
        Kc[M.off_Kc + e] = v;
    }
}

// MFMA operand layouts of the augmented operator A_s = [F_s; F_rc^T] (rows_F x ldF):
//  FP64 / FP32 (16x16x4 MFMA): element ((rb*KQ + kq)*64 + lane)*4 + q holds
//      A[16 rb + lane%16][16 kq + 4 q + lane/16],  KQ = ldF/16;
//  BF16 (16x16x32 MFMA): element ((rb*KB + kb)*64 + lane)*8 + q holds
//      A[16 rb + lane%16][32 kb + 8 (lane/16) + q],  KB = ldF/32;
// stored as a hi part (round to nearest) and a lo part (the rounded remainder).
__global__ void k_swizzle(const SubMeta* __restrict__ subs, const double* __restrict__ F64, double* sw64,
                          float* sw32, __hip_bfloat16* swhi, __hip_bfloat16* swlo) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const long long tot = (long long)M.rows_F * M.ldF;
    const int KQ = M.ldF / 16, KB = M.ldF / 32;
    auto live = [&](int row) { return row < M.n_b || (row >= M.rowT && row < M.rowT + M.n_c); };
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
        {
            const int q = (int)(e & 3), lane = (int)((e >> 2) & 63);
            const long long blk = e >> 8;
            const int rb = (int)(blk / KQ), kq = (int)(blk % KQ);
            const int row = 16 * rb + (lane & 15), col = 16 * kq + 4 * q + (lane >> 4);
            const double v = (live(row) && col < M.n_b) ? F64[M.off_F + (long long)row * M.ldF + col] : 0.0;
            sw64[M.off_Fsw + e] = v;
            sw32[M.off_Fsw + e] = (float)v;
        }
        {
            // lane operand e = 4h + q of the 16x16x32 MFMA takes contraction index
            // 32 kb + 16 h + 4 q + lane/16: the same permutation is applied to X_s, whose
            // FP64 operand order then serves the BF16 products without a lane exchange
            const int q = (int)(e & 7), lane = (int)((e >> 3) & 63);
            const long long blk = e >> 9;
            const int rb = (int)(blk / KB), kb = (int)(blk % KB);
            const int row = 16 * rb + (lane & 15), col = 32 * kb + 16 * (q >> 2) + 4 * (q & 3) + (lane >> 4);
            const double v = (live(row) && col < M.n_b) ? F64[M.off_F + (long long)row * M.ldF + col] : 0.0;
            const float vf = (float)v;
            const __hip_bfloat16 hi = __float2bfloat16(vf);
            const __hip_bfloat16 lo = __float2bfloat16(vf - __bfloat162float(hi));
            swhi[M.off_Fsw + e] = hi;
            swlo[M.off_Fsw + e] = lo;
        }
    }
}

// ---------------------------------------------------------------------------------------
// Scaling weights (Sec. 3.1): per lambda row and side. Dirichlet rows: 1. Multiplicity:
// 1/m. k-scaling (Eq. 15, multi-domain form): the weight of side a is K^b_jj / sum_q K^q_jj
// with the sum over every subdomain sharing the DOF.
__global__ void k_weights(int n_lambda, int kscale, const int* __restrict__ row_s, const int* __restrict__ row_j,
                          const int* __restrict__ row_sh, const int* __restrict__ sh_ptr,
                          const int* __restrict__ sh_s, const int* __restrict__ sh_l,
                          const SubMeta* __restrict__ subs, const int* __restrict__ b_loc,
                          const double* __restrict__ diag, double* w) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_lambda) return;
    const int sh = row_sh[r];
    if (sh < 0) {
        w[2 * r] = 1.0;
        w[2 * r + 1] = 0.0;
        return;
    }
    const int m = sh_ptr[sh + 1] - sh_ptr[sh];
    if (!kscale) {
        w[2 * r] = 1.0 / m;
        w[2 * r + 1] = 1.0 / m;
        return;
    }
    double tot = 0.0;
    for (int q = sh_ptr[sh]; q < sh_ptr[sh + 1]; ++q) tot += diag[subs[sh_s[q]].off_loc + sh_l[q]];
    double dside[2];
    for (int t = 0; t < 2; ++t) {
        const int s = row_s[2 * r + t];
        const SubMeta& M = subs[s];
        dside[t] = diag[M.off_loc + b_loc[M.off_b + row_j[2 * r + t]]];
    }
    w[2 * r] = dside[1] / tot;
    w[2 * r + 1] = dside[0] / tot;
}

// Weight of every gather entry (b DOF, row): the weight of the b DOF's own side of the row.
__global__ void k_bg_weights(long long nb_tot, const int* __restrict__ bq_s, const SubMeta* __restrict__ subs,
                             const int* __restrict__ bg_ptr, const int* __restrict__ bg_row,
                             const int* __restrict__ row_s, const int* __restrict__ row_j,
                             const double* __restrict__ w, double* bg_w) {
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= nb_tot) return;
    const int s = bq_s[q];
    const int j = (int)(q - subs[s].off_b);
    for (int e = bg_ptr[q]; e < bg_ptr[q + 1]; ++e) {
        const int r = bg_row[e];
        const int t = (row_s[2 * r] == s && row_j[2 * r] == j) ? 0 : 1;
        bg_w[e] = w[2 * r + t];
    }
}

// Coarse matrix Kbar_cc = sum_s B_c^sT Kbar_cc^s B_c^s (Sec. 2.2), one thread per global
// corner row (owner computes, fixed summation order).
// Row p of Kbar_cc, inside its design's dense block (corners of one design couple only among
// themselves): one thread per corner, each entry written by its row's thread only.
__global__ void k_coarse_assemble(int n_cg, const int* __restrict__ cc_ptr, const int* __restrict__ cc_s,
                                  const int* __restrict__ cc_j, const SubMeta* __restrict__ subs,
                                  const int* __restrict__ c_glob, const int* __restrict__ cg_blk,
                                  const CoarseBlk* __restrict__ blks, const double* __restrict__ Kc, double* Kg) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_cg) return;
    const CoarseBlk B = blks[cg_blk[p]];
    double* row = Kg + B.off + (long long)(p - B.cg0) * B.n - B.cg0;
    for (int e = cc_ptr[p]; e < cc_ptr[p + 1]; ++e) {
        const int s = cc_s[e], jc = cc_j[e];
        const SubMeta& M = subs[s];
        for (int c2 = 0; c2 < M.n_c; ++c2) row[c_glob[M.off_c + c2]] += Kc[M.off_Kc + jc * M.n_c + c2];
    }
}

// TFETI: G G^T with G = -Rhat^T B^T, one thread per subdomain owning its rows of G G^T.
__global__ void k_ggt_assemble(int n_sub, int nm, const SubMeta* __restrict__ subs, const int* __restrict__ bg_ptr,
                               const int* __restrict__ bg_row, const int8_t* __restrict__ bg_sg,
                               const int* __restrict__ row_s, const int* __restrict__ row_j,
                               const int8_t* __restrict__ row_sg, const double* __restrict__ Rb, double* GG) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sub) return;
    const SubMeta M = subs[s];
    const int na = n_sub * nm;
    for (int j = 0; j < M.n_b; ++j) {
        const long long q = M.off_b + j;
        for (int e = bg_ptr[q]; e < bg_ptr[q + 1]; ++e) {
            const int r = bg_row[e];
            const double sg = bg_sg[e];
            for (int t = 0; t < 2; ++t) {
                const int s2 = row_s[2 * r + t];
                if (s2 < 0) continue;
                const SubMeta& M2 = subs[s2];
                const int j2 = row_j[2 * r + t];
                const double sg2 = row_sg[2 * r + t];
                for (int m = 0; m < nm; ++m)
                    for (int m2 = 0; m2 < nm; ++m2)
                        GG[(long long)(s * nm + m) * na + s2 * nm + m2] +=
                            sg * sg2 * Rb[M.off_R + (long long)j * nm + m] * Rb[M2.off_R + (long long)j2 * nm + m2];
            }
        }
    }
}

// dst[s] = round_P(F_s), leading n_b x n_b block of the augmented operator, ld n_b.
__global__ void k_copy_F_rounded(const SubMeta* __restrict__ subs, const double* __restrict__ F64, int precision,
                                 double* dst) {
    const int s = blockIdx.y;
    const SubMeta M = subs[s];
    const long long nn = (long long)M.n_b * M.n_b;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn; e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / M.n_b), j = (int)(e % M.n_b);
        const double v = F64[M.off_F + (long long)i * M.ldF + j];
        double r = v;
        if (precision == FETI_FP32) {
            r = (double)(float)v;
        } else if (precision == FETI_BF16X3) {
            const float vf = (float)v;
            const float hi = __bfloat162float(__float2bfloat16(vf));
            const float lo = __bfloat162float(__float2bfloat16(vf - hi));
            r = (double)hi + (double)lo;
        }
        dst[M.off_P + e] = r;
    }
}

// Per-subdomain round-off test: largest relative change of a Cholesky pivot.
__global__ void k_pivot_compare(const SubMeta* __restrict__ subs, const double* __restrict__ W1,
                                const double* __restrict__ W2, const int* __restrict__ info2, double* dev) {
    __shared__ double red[256];
    const int s = blockIdx.x;
    const SubMeta M = subs[s];
    double m = 0.0;
    for (int j = threadIdx.x; j < M.n_b; j += 256) {
        const double a = W1[M.off_P + (long long)j * M.n_b + j], b = W2[M.off_P + (long long)j * M.n_b + j];
        const double r = fabs((b * b) / (a * a) - 1.0);
        m = fmax(m, r == r ? r : 1e300);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int u = 0; u < 256; ++u) v = fmax(v, red[u]);
        dev[s] = info2[s] ? 1e300 : v;
    }
}

__global__ void k_set_identity(double* A, int n, long long lda) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)n * n) return;
    const int i = (int)(e / n), j = (int)(e % n);
    A[(long long)i * lda + j] = i == j ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------------------
// host launchers

// ---- module types (factorisation recycling) ----
// Element e of subdomain s in local lexicographic order (x fastest), as its global index.
__device__ __forceinline__ long long sub_element(const SubMeta& M, int dim, int e) {
    const int nx = M.nn[0] - 1, ny = M.nn[1] - 1;
    const int ex = e % nx, ey = (e / nx) % ny, ez = dim == 3 ? e / (nx * ny) : 0;
    return M.el0 + (long long)(M.lo[0] + ex) + (long long)M.nelx * ((M.lo[1] + ey) + (long long)M.nely * (M.lo[2] + ez));
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// out[s] = XOR over the subdomain's elements of mix64(bits(rho_e) + mix64(local index)): equal
// density patterns give equal values (order-independent, so deterministic); unequal ones almost
// surely do not, and the host checks candidates element by element (k_rho_match).
__global__ void __launch_bounds__(256) k_rho_hash(const SubMeta* __restrict__ subs, int dim, const double* __restrict__ rho,
                                                  unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[4];
    const SubMeta M = subs[blockIdx.x];
    const int nel = (M.nn[0] - 1) * (M.nn[1] - 1) * (dim == 3 ? M.nn[2] - 1 : 1);
    unsigned long long h = 0;
    for (int e = threadIdx.x; e < nel; e += 256)
        h ^= mix64((unsigned long long)__double_as_longlong(rho[sub_element(M, dim, e)]) + mix64((unsigned long long)e));
    for (int o = 32; o > 0; o >>= 1) h ^= __shfl_xor(h, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = h;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = red[0] ^ red[1] ^ red[2] ^ red[3];
}

// flag[q] = 1 if the densities of subdomain pairs[2q] differ anywhere from those of pairs[2q+1]
// (same local layout), else 0
__global__ void __launch_bounds__(256) k_rho_match(const SubMeta* __restrict__ subs, int dim, const double* __restrict__ rho,
                                                   const int* __restrict__ pairs, int* __restrict__ flag) {
    __shared__ int any;
    const SubMeta A = subs[pairs[2 * blockIdx.x]], B = subs[pairs[2 * blockIdx.x + 1]];
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    const int nel = (A.nn[0] - 1) * (A.nn[1] - 1) * (dim == 3 ? A.nn[2] - 1 : 1);
    int d = 0;
    for (int e = threadIdx.x; e < nel; e += 256)
        d |= __double_as_longlong(rho[sub_element(A, dim, e)]) != __double_as_longlong(rho[sub_element(B, dim, e)]);
    if (d) any = 1;
    __syncthreads();
    if (threadIdx.x == 0) flag[blockIdx.x] = any;
}

// dst[i * w + j] = src[map[i] * w + j], i < n
__global__ void k_gather_rows(int n, int w, const int* __restrict__ map, const double* __restrict__ src,
                              double* __restrict__ dst) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)n * w) return;
    const int i = (int)(e / w), j = (int)(e % w);
    dst[e] = src[(long long)map[i] * w + j];
}

void launch_rho_hash(const DevTopo& t, const double* rho, unsigned long long* out, hipStream_t st) {
    if (t.n_sub) k_rho_hash<<<t.n_sub, 256, 0, st>>>(t.subs, t.dim, rho, out);
}

void launch_rho_match(const DevTopo& t, const double* rho, const int* pairs, int npairs, int* flag, hipStream_t st) {
    if (npairs) k_rho_match<<<npairs, 256, 0, st>>>(t.subs, t.dim, rho, pairs, flag);
}

void launch_gather_rows(int n, int w, const int* map, const double* src, double* dst, hipStream_t st) {
    const long long m = (long long)n * w;
    if (m) k_gather_rows<<<(int)((m + 255) / 256), 256, 0, st>>>(n, w, map, src, dst);
}

void launch_assemble(const DevTopo& t, const double* Emod, double* L, double* Z, double* S, double* diag,
                     hipStream_t st) {
    dim3 grid((t.max_nodes + 255) / 256, t.n_sub);
    k_assemble<<<grid, 256, 0, st>>>(t.subs, t.lines, t.dim, t.K0dev, Emod, t.lcls, t.lidx, L, Z, S, diag);
}

size_t bt_plane_ws_bytes(const DevTopo& t) {
    return (size_t)t.max_planes * t.n_sub * (sizeof(PotrfDesc) + sizeof(int));
}

void launch_bt_factor(const DevTopo& t, double* L, int* info, void* ws, hipStream_t st) {
    const int ns = t.n_sub, np = t.max_planes;
    if (ns == 0) return;
    PotrfDesc* pd = static_cast<PotrfDesc*>(ws);
    int* pinfo = reinterpret_cast<int*>(pd + (size_t)np * ns);
    if (np > 0) k_plane_descs<<<(np * ns + 255) / 256, 256, 0, st>>>(t.subs, ns, t.lines, np, pd, pinfo);
    const int nb = (t.max_line + 63) / 64;
    for (int k = 0; k < np; ++k) {
        if (k > 0 && nb > 0) k_plane_syrk<<<dim3(nb * (nb + 1) / 2, ns), 256, 0, st>>>(t.subs, t.lines, k, L);
        launch_potrf(pd + (size_t)k * ns, ns, t.max_line, L, pinfo + (size_t)k * ns, st);
        if (k + 1 < np && nb > 0) k_plane_trsm<<<dim3(nb, ns), 256, 0, st>>>(t.subs, t.lines, k, L);
    }
    k_plane_info<<<(ns + 255) / 256, 256, 0, st>>>(t.subs, ns, t.lines, np, pinfo, info);
}

void launch_bt_forward(const DevTopo& t, const double* L, double* Z, hipStream_t st) {
    dim3 grid((t.max_beta + 63) / 64, t.n_sub);
    k_bt_forward<<<grid, 256, 0, st>>>(t.subs, t.lines, L, Z);
}

// FP64 MFMA factorisation with the inverses for lines <= 128 DOFs, else the generic path
// followed by the separate inverse kernel
void launch_bt_factor_li(const DevTopo& t, double* L, double* Li, int* info, void* ws, hipStream_t st) {
    if (t.max_line <= 128) {
        if (t.n_sub) k_bt_factor128<<<t.n_sub, 256, 0, st>>>(t.subs, t.lines, L, Li, info);
        return;
    }
    launch_bt_factor(t, L, info, ws, st);
}

long long bt_plane_fwd_doubles(const DevTopo& t) {
    return (long long)t.max_line * t.max_beta * t.n_sub;
}

void launch_bt_forward_planes(const DevTopo& t, const double* L, const double* Li, double* Z, double* T,
                              hipStream_t st) {
    const int ntr = (t.max_line + 63) / 64, ntc = (t.max_beta + 63) / 64;
    if (t.n_sub == 0 || ntr == 0 || ntc == 0) return;
    const long long ts = (long long)t.max_line * t.max_beta;
    for (int k = 0; k < t.max_planes; ++k) {
        k_plane_fwd<0><<<dim3(ntr * ntc, t.n_sub), 256, 0, st>>>(t.subs, t.lines, k, ntr, L, Li, Z, T, ts);
        k_plane_fwd<1><<<dim3(ntr * ntc, t.n_sub), 256, 0, st>>>(t.subs, t.lines, k, ntr, L, Li, Z, T, ts);
    }
}

void launch_bt_forward_li(const DevTopo& t, const double* L, const double* Li, double* Z, hipStream_t st) {
    if (t.max_line > 128) {
        launch_bt_forward(t, L, Z, st);
        return;
    }
    if (t.n_sub && t.max_beta) k_bt_forward_mfma<<<dim3((t.max_beta + 63) / 64, t.n_sub), 256, 0, st>>>(t.subs, t.lines, L, Li, Z);
}

void launch_gemm_tn(const GemmDesc* d, int nbatch, int tdim, const double* A, const double* B, double* C,
                    double alpha, double beta, int symmetric, hipStream_t st) {
    if (nbatch == 0 || tdim == 0) return;
    const int tiles = symmetric ? tdim * (tdim + 1) / 2 : tdim * tdim;
    k_gemm_tn<<<dim3(tiles, 8 * ((nbatch + 7) / 8)), 256, 0, st>>>(d, nbatch, A, B, C, alpha, beta, symmetric);
}

void launch_potrf(const PotrfDesc* d, int nbatch, int max_n, double* base, int* info, hipStream_t st) {
    if (nbatch == 0) return;
    if (max_n <= 512) {   // one workgroup per matrix
        k_potrf512<<<nbatch, 512, 0, st>>>(d, base, info);
        return;
    }
    // panels in pairs: the first panel's update of the second panel's columns, then one pass of
    // both over the trailing matrix (half the passes of a panel-by-panel update)
    for (int p0 = 0; p0 < max_n; p0 += 2 * kPfB) {
        k_potrf_diag<<<nbatch, 256, 0, st>>>(d, p0, base, info);
        const int rest = max_n - p0 - kPfB;
        if (rest <= 0) break;
        k_potrf_panel<<<dim3((rest + kPfRows - 1) / kPfRows, nbatch), 256, 0, st>>>(d, p0, base, info);
        k_potrf_syrk<<<dim3((rest + 63) / 64, nbatch), 256, 0, st>>>(d, p0, kPfB, 1, base, info);
        k_potrf_diag<<<nbatch, 256, 0, st>>>(d, p0 + kPfB, base, info);
        const int rest2 = rest - kPfB;
        if (rest2 <= 0) break;
        k_potrf_panel<<<dim3((rest2 + kPfRows - 1) / kPfRows, nbatch), 256, 0, st>>>(d, p0 + kPfB, base, info);
        const int nt = (rest2 + 63) / 64;
        k_potrf_syrk<<<dim3(nt * (nt + 1) / 2, nbatch), 256, 0, st>>>(d, p0, 2 * kPfB, 0, base, info);
    }
}

void launch_trsm_identity(const TrsmDesc* d, int nbatch, int max_cols, const double* L, double* B, hipStream_t st) {
    if (nbatch && max_cols) k_trsm<<<dim3((max_cols + 63) / 64, nbatch), 256, 0, st>>>(d, L, B);
}

void launch_copy_Sbb(const DevTopo& t, const double* S, double* dst, int identity, hipStream_t st) {
    k_copy_Sbb<<<dim3(64, t.n_sub), 256, 0, st>>>(t.subs, S, dst, identity);
}

void launch_pack_sym(const DevTopo& t, const double* S, double* Pk, hipStream_t st) {
    k_pack_sym<<<dim3(64, t.n_sub), 256, 0, st>>>(t.subs, S, Pk);
}

void launch_tfeti_rbm(const DevTopo& t, const double* S, double* Rb, double* Cit, double* tau, double* W,
                      hipStream_t st) {
    k_tfeti_rbm<<<t.n_sub, 256, 0, st>>>(t.subs, t.dim, t.b_loc, S, Rb, Cit, tau, W);
}

void launch_tfeti_fix(const DevTopo& t, const double* Rb, const double* tau, double* F64, hipStream_t st) {
    k_tfeti_fix<<<dim3(64, t.n_sub), 256, 0, st>>>(t.subs, t.dim == 2 ? 3 : 6, Rb, tau, F64);
}

void launch_frc(const DevTopo& t, const double* S, double* F64, double* Kc, hipStream_t st) {
    if (t.n_sub == 0 || t.max_nb == 0) return;
    k_frc<<<dim3((t.max_nb + 255) / 256, t.n_sub), 256, 0, st>>>(t.subs, S, F64);
    k_frc_kc<<<t.n_sub, 256, 0, st>>>(t.subs, S, F64, Kc);
}

void launch_swizzle(const DevTopo& t, const double* F64, double* sw64, float* sw32, __hip_bfloat16* hi,
                    __hip_bfloat16* lo, hipStream_t st) {
    k_swizzle<<<dim3(256, t.n_sub), 256, 0, st>>>(t.subs, F64, sw64, sw32, hi, lo);
}

void launch_weights(const DevTopo& t, int kscale, const double* diag, double* w, double* bg_w, hipStream_t st) {
    if (t.n_lambda == 0) return;
    k_weights<<<(t.n_lambda + 255) / 256, 256, 0, st>>>(t.n_lambda, kscale, t.row_s, t.row_j, t.row_sh, t.sh_ptr,
                                                         t.sh_s, t.sh_l, t.subs, t.b_loc, diag, w);
    k_bg_weights<<<(int)((t.nb_tot + 255) / 256), 256, 0, st>>>(t.nb_tot, t.bq_s, t.subs, t.bg_ptr, t.bg_row,
                                                                 t.row_s, t.row_j, w, bg_w);
}

void launch_coarse_assemble(const DevTopo& t, const double* Kc, double* Kg, hipStream_t st) {
    if (t.n_cg) k_coarse_assemble<<<(t.n_cg + 255) / 256, 256, 0, st>>>(t.n_cg, t.cc_ptr, t.cc_s, t.cc_j, t.subs,
                                                                          t.c_glob, t.cg_blk, t.cblk, Kc, Kg);
}

void launch_ggt_assemble(const DevTopo& t, const double* Rb, double* GG, hipStream_t st) {
    k_ggt_assemble<<<(t.n_sub + 63) / 64, 64, 0, st>>>(t.n_sub, t.dim == 2 ? 3 : 6, t.subs, t.bg_ptr, t.bg_row,
                                                       t.bg_sg, t.row_s, t.row_j, t.row_sg, Rb, GG);
}

void launch_copy_F_rounded(const DevTopo& t, const double* F64, int precision, double* dst, hipStream_t st) {
    k_copy_F_rounded<<<dim3(64, t.n_sub), 256, 0, st>>>(t.subs, F64, precision, dst);
}

void launch_pivot_compare(const DevTopo& t, const double* W1, const double* W2, const int* info2, double* dev,
                          hipStream_t st) {
    k_pivot_compare<<<t.n_sub, 256, 0, st>>>(t.subs, W1, W2, info2, dev);
}

void launch_set_identity(double* A, int n, long long lda, hipStream_t st) {
    if (n) k_set_identity<<<(int)(((long long)n * n + 255) / 256), 256, 0, st>>>(A, n, lda);
}

}  // namespace feti
