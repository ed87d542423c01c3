// Deflation of local interface modes (Sec. 6, item (ii): the interface modes responsible for slow
// convergence are identified by local eigenproblems, in the manner of GenEO, and removed from the
// iteration). Per subdomain s, with F_s = L L^T its interface block of the dual operator, S~ its
// preconditioner block and omega the summed weights of each interface DOF over its dual rows:
//     C_s = L^T (omega S~ omega) L        (symmetric; its eigenvalues are the nonzero ones of the
//                                          local preconditioned operator P_s F_s)
// and for C_s x = mu x the dual vector y = diag(w_s) B_s u, u = omega^{-1} (omega S~ omega) L x.
// The largest eigenpairs come from a subspace iteration of 16 vectors (orthonormalised by
// Cholesky QR, twice) and a Rayleigh-Ritz step; of them the k <= m leading ones that end at a
// relative spectral gap (mu_k >= (1 + gap) mu_{k+1}) and lie above tau are taken.
#include "kernels.hpp"

namespace feti {

namespace {
typedef double v4x __attribute__((ext_vector_type(4)));
constexpr int kP = kDeflSubspace;   // subspace width (16)
constexpr int kGs = 17;             // stride of the 16 x 16 LDS matrices

// deterministic start vector entry in [-0.5, 0.5) (a 32-bit integer hash of the position)
__device__ inline double start_entry(int j, int c) {
    unsigned x = (unsigned)(j * kP + c) * 2654435761u + 0x9e3779b9u;
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return (double)(x >> 8) * (1.0 / 16777216.0) - 0.5;
}

// out = A in for the n x n row-major A (global) and in (np x 16, LDS, rows n .. np-1 zero), on the
// FP64 matrix cores; wavefront w computes the 16-row blocks w, w + 4, ... Eight k-steps of A are
// loaded ahead of their products.
__device__ void apply_block(const double* __restrict__ A, int n, int np, const double* in, double* out) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, m = lane & 15, g = lane >> 4;
    const int nq = np >> 4;
    for (int I = wave; I < nq; I += 4) {
        v4x acc = v4x{0.0, 0.0, 0.0, 0.0};
        const int r = 16 * I + m;
        const double* Ar = A + (long long)min(r, n - 1) * n;
        for (int Q0 = 0; Q0 < nq; Q0 += 8) {
            double a[8][4];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int q = 16 * (Q0 + u) + 4 * kk + g;
                    a[u][kk] = (r < n && q < n) ? Ar[q] : 0.0;
                }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (Q0 + u < nq) {
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][kk], in[(16 * (Q0 + u) + 4 * kk + g) * kP + m],
                                                                   acc, 0, 0, 0);
                }
            }
        }
        // D layout: rows g + 4v, column m
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(16 * I + g + 4 * v) * kP + m] = acc[v];
    }
}

// V (rows < n) <- V R^{-1} with V^T V = R^T R; G: LDS scratch. The Gram matrix gets a relative
// diagonal shift of 1e-14 against rank loss at round-off level (the span is unchanged, and the
// second pass of the caller restores orthonormality).
__device__ void cholqr(double* V, int n, double* G) {
    const int tid = threadIdx.x;
    {
        const int a = tid >> 4, b = tid & 15;
        double s = 0.0;
        for (int j = 0; j < n; ++j) s = fma(V[j * kP + a], V[j * kP + b], s);
        G[a * kGs + b] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double tr = 0.0;
        for (int a = 0; a < kP; ++a) tr += G[a * kGs + a];
        for (int a = 0; a < kP; ++a) G[a * kGs + a] += 1e-14 * tr;
        for (int k = 0; k < kP; ++k) {   // G = R^T R, R in the upper triangle
            double d = G[k * kGs + k];
            for (int q = 0; q < k; ++q) d -= G[q * kGs + k] * G[q * kGs + k];
            d = sqrt(fmax(d, 1e-300));
            G[k * kGs + k] = d;
            for (int j = k + 1; j < kP; ++j) {
                double v = G[k * kGs + j];
                for (int q = 0; q < k; ++q) v -= G[q * kGs + k] * G[q * kGs + j];
                G[k * kGs + j] = v / d;
            }
        }
    }
    __syncthreads();
    for (int j = tid; j < n; j += 256) {
        double x[kP];
#pragma unroll
        for (int c = 0; c < kP; ++c) {
            double v = V[j * kP + c];
#pragma unroll
            for (int a = 0; a < c; ++a) v -= x[a] * G[a * kGs + c];
            x[c] = v / G[c * kGs + c];
        }
#pragma unroll
        for (int c = 0; c < kP; ++c) V[j * kP + c] = x[c];
    }
    __syncthreads();
}

// H (16 x 16, symmetric, stride kGs) = U diag(th) U^T by cyclic Jacobi rotations (one thread);
// th sorted in decreasing order with the columns of U.
__device__ void jacobi16(double* H, double* U, double* th) {
    for (int i = 0; i < kP; ++i)
        for (int j = 0; j < kP; ++j) U[i * kGs + j] = i == j ? 1.0 : 0.0;
    double fro = 0.0;
    for (int i = 0; i < kP; ++i)
        for (int j = 0; j < kP; ++j) fro += H[i * kGs + j] * H[i * kGs + j];
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < kP; ++p)
            for (int q = p + 1; q < kP; ++q) off += H[p * kGs + q] * H[p * kGs + q];
        if (!(off > 1e-32 * fro)) break;
        for (int p = 0; p < kP; ++p)
            for (int q = p + 1; q < kP; ++q) {
                const double apq = H[p * kGs + q];
                if (apq == 0.0) continue;
                const double theta = (H[q * kGs + q] - H[p * kGs + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < kP; ++k) {   // columns p, q
                    const double hp = H[k * kGs + p], hq = H[k * kGs + q];
                    H[k * kGs + p] = c * hp - s * hq;
                    H[k * kGs + q] = s * hp + c * hq;
                    const double up = U[k * kGs + p], uq = U[k * kGs + q];
                    U[k * kGs + p] = c * up - s * uq;
                    U[k * kGs + q] = s * up + c * uq;
                }
                for (int k = 0; k < kP; ++k) {   // rows p, q
                    const double hp = H[p * kGs + k], hq = H[q * kGs + k];
                    H[p * kGs + k] = c * hp - s * hq;
                    H[q * kGs + k] = s * hp + c * hq;
                }
            }
    }
    for (int i = 0; i < kP; ++i) th[i] = H[i * kGs + i];
    for (int i = 0; i < kP; ++i) {   // selection sort, decreasing
        int b = i;
        for (int j = i + 1; j < kP; ++j)
            if (th[j] > th[b]) b = j;
        if (b != i) {
            const double tt = th[i];
            th[i] = th[b];
            th[b] = tt;
            for (int k = 0; k < kP; ++k) {
                const double uu = U[k * kGs + i];
                U[k * kGs + i] = U[k * kGs + b];
                U[k * kGs + b] = uu;
            }
        }
    }
}
}  // namespace

// omega[q] = sum of the weights (its subdomain's side) of the dual rows of interface DOF q
__global__ void k_defl_omega(long long nb_tot, const int* __restrict__ bg_ptr, const double* __restrict__ bg_w,
                             double* __restrict__ omega) {
    const long long q = blockIdx.x * 256LL + threadIdx.x;
    if (q >= nb_tot) return;
    double s = 0.0;
    for (int e = bg_ptr[q]; e < bg_ptr[q + 1]; ++e) s += bg_w[e];
    omega[q] = s;
}

// DL = F_s (interface block of the dual operator, for its Cholesky factor) and
// DM = omega S~ omega, both n_b x n_b row-major at off_P
__global__ void __launch_bounds__(256) k_defl_prep(const SubMeta* __restrict__ subs, const double* __restrict__ F64,
                                                   const double* __restrict__ Pk, const double* __restrict__ omega,
                                                   double* __restrict__ DL, double* __restrict__ DM) {
    const SubMeta M = subs[blockIdx.y];
    const int nb = M.n_b;
    const long long tot = (long long)nb * nb;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
        const int i = (int)(e / nb), j = (int)(e - (long long)i * nb);
        DL[M.off_P + e] = F64[M.off_F + (long long)i * M.ldF + j];
        const int a = min(i, j), b = max(i, j), I = a >> 6, J = b >> 6;
        const double sv = Pk[M.off_Pk + ((long long)J * (J + 1) / 2 + I) * 4096 + (a & 63) * 64 + (b & 63)];
        DM[M.off_P + e] = omega[M.off_b + i] * sv * omega[M.off_b + j];
    }
}

// the strict upper triangle of the Cholesky factors to zero (the factorisation leaves it unspecified)
__global__ void __launch_bounds__(256) k_defl_tril(const SubMeta* __restrict__ subs, double* __restrict__ DL) {
    const SubMeta M = subs[blockIdx.y];
    const int nb = M.n_b;
    const long long tot = (long long)nb * nb;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
        const int i = (int)(e / nb), j = (int)(e - (long long)i * nb);
        if (j > i) DL[M.off_P + e] = 0.0;
    }
}

// One workgroup per subdomain: the largest eigenpairs of C_s (DC, n_b x n_b at off_P) and
// u = omega^{-1} DB x (DB = (omega S~ omega) L at off_P). Writes U[(off_b + j) * 8 + i] (i < 8, zero
// past the k selected), mu[s * m + i] (zero past k) and cnt[s] = k. Subdomains whose n_b lies
// outside [2 * 16, kDeflMaxNb] take no modes.
__global__ void __launch_bounds__(256) k_defl_eig(const SubMeta* __restrict__ subs, const double* __restrict__ DC,
                                                  const double* __restrict__ DB, const double* __restrict__ omega,
                                                  int m, double tau, double gap, int n_it, double* __restrict__ U,
                                                  double* __restrict__ mu, int* __restrict__ cnt) {
    __shared__ double V[kDeflMaxNb * kP];
    __shared__ double X[kDeflMaxNb * kP];
    __shared__ double G[kP * kGs];
    __shared__ double Uh[kP * kGs];
    __shared__ double th[kP];
    __shared__ int ksel;
    const int s = blockIdx.x, tid = threadIdx.x;
    const SubMeta M = subs[s];
    const int n = M.n_b, np = (n + 15) & ~15;
    if (n < 2 * kP || n > kDeflMaxNb) {
        for (int j = tid; j < n * 8; j += 256) U[M.off_b * 8 + j] = 0.0;
        if (tid < m) mu[(long long)s * m + tid] = 0.0;
        if (tid == 0) cnt[s] = 0;
        return;
    }
    const double* C = DC + M.off_P;
    const double* B = DB + M.off_P;
    for (int e = tid; e < np * kP; e += 256) {
        const int j = e / kP, c = e - j * kP;
        V[e] = j < n ? start_entry(j, c) : 0.0;
        X[e] = 0.0;
    }
    __syncthreads();
    cholqr(V, n, G);
    cholqr(V, n, G);
    for (int it = 0; it < n_it; ++it) {
        apply_block(C, n, np, V, X);
        __syncthreads();
        for (int e = tid; e < np * kP; e += 256) V[e] = X[e];
        __syncthreads();
        cholqr(V, n, G);
        cholqr(V, n, G);
    }
    // Rayleigh-Ritz: H = V^T C V
    apply_block(C, n, np, V, X);
    __syncthreads();
    {
        const int a = tid >> 4, b = tid & 15;
        double sacc = 0.0;
        for (int j = 0; j < n; ++j) sacc = fma(V[j * kP + a], X[j * kP + b], sacc);
        Uh[a * kGs + b] = sacc;
    }
    __syncthreads();
    if (tid == 0) {
        for (int a = 0; a < kP; ++a)
            for (int b = 0; b < kP; ++b) G[a * kGs + b] = 0.5 * (Uh[a * kGs + b] + Uh[b * kGs + a]);
        jacobi16(G, Uh, th);
        int k = 0;
        for (int kk = min(m, kP - 1); kk > 0 && k == 0; --kk)
            if (th[kk - 1] >= tau && th[kk - 1] >= (1.0 + gap) * th[kk]) k = kk;
        ksel = k;
    }
    __syncthreads();
    const int k = ksel;
    // X = V Uh[:, :k] (Ritz vectors), then V = DB X, u = omega^{-1} V
    for (int j = tid; j < np; j += 256) {
        double x[kP];
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            double acc = 0.0;
            if (i < k && j < n)
                for (int c = 0; c < kP; ++c) acc = fma(V[j * kP + c], Uh[c * kGs + i], acc);
            x[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < kP; ++i) X[j * kP + i] = x[i];
    }
    __syncthreads();
    apply_block(B, n, np, X, V);
    __syncthreads();
    for (int e = tid; e < n * 8; e += 256) {
        const int j = e >> 3, i = e & 7;
        U[(M.off_b + j) * 8 + i] = i < k ? V[j * kP + i] / omega[M.off_b + j] : 0.0;
    }
    if (tid < m) mu[(long long)s * m + tid] = tid < k ? th[tid] : 0.0;
    if (tid == 0) cnt[s] = k;
}

// Y (blocks of n_lambda x 64, row-major, zeroed before) column col0[s] + i of subdomain s's mode i:
// y_r = w_r sign_r u_j for every dual row r of its interface DOF j
__global__ void k_defl_scatter(long long nb_tot, int n_lambda, const int* __restrict__ bq_s,
                               const int* __restrict__ bg_ptr, const int* __restrict__ bg_row,
                               const int8_t* __restrict__ bg_sg, const double* __restrict__ bg_w,
                               const double* __restrict__ U, const int* __restrict__ col0,
                               const int* __restrict__ cnt, double* __restrict__ Y) {
    const long long q = blockIdx.x * 256LL + threadIdx.x;
    if (q >= nb_tot) return;
    const int s = bq_s[q], k = cnt[s], c0 = col0[s];
    for (int e = bg_ptr[q]; e < bg_ptr[q + 1]; ++e) {
        const long long r = bg_row[e];
        const double f = bg_w[e] * (double)bg_sg[e];
        for (int i = 0; i < k; ++i) {
            const int col = c0 + i;
            Y[(long long)(col >> 6) * n_lambda * 64 + r * 64 + (col & 63)] = f * U[q * 8 + i];
        }
    }
}

// the first kd columns of the n x 64 block P from the n x kd block Z (dir 0), or back (dir 1)
__global__ void k_pad64(int n, int kd, int dir, double* __restrict__ Z, double* __restrict__ P) {
    const long long e = blockIdx.x * 256LL + threadIdx.x;
    if (e >= (long long)n * kd) return;
    const long long r = e / kd, c = e - r * kd;
    if (dir == 0)
        P[r * 64 + c] = Z[e];
    else
        Z[e] = P[r * 64 + c];
}

void launch_defl_local(const DevTopo& t, const double* F64, const double* Pk, const double* bg_w, double* omega,
                       double* DL, double* DM, hipStream_t st) {
    if (t.nb_tot == 0) return;
    k_defl_omega<<<(int)((t.nb_tot + 255) / 256), 256, 0, st>>>(t.nb_tot, t.bg_ptr, bg_w, omega);
    k_defl_prep<<<dim3(64, t.n_sub), 256, 0, st>>>(t.subs, F64, Pk, omega, DL, DM);
}

void launch_defl_tril(const DevTopo& t, double* DL, hipStream_t st) {
    if (t.n_sub) k_defl_tril<<<dim3(64, t.n_sub), 256, 0, st>>>(t.subs, DL);
}

void launch_defl_eig(const DevTopo& t, const double* DC, const double* DB, const double* omega, int m, double tau,
                     double gap, int n_it, double* U, double* mu, int* cnt, hipStream_t st) {
    if (t.n_sub) k_defl_eig<<<t.n_sub, 256, 0, st>>>(t.subs, DC, DB, omega, m, tau, gap, n_it, U, mu, cnt);
}

void launch_defl_scatter(const DevTopo& t, const double* bg_w, const double* U, const int* col0, const int* cnt,
                         double* Y, hipStream_t st) {
    if (t.nb_tot)
        k_defl_scatter<<<(int)((t.nb_tot + 255) / 256), 256, 0, st>>>(t.nb_tot, t.n_lambda, t.bq_s, t.bg_ptr, t.bg_row,
                                                                       t.bg_sg, bg_w, U, col0, cnt, Y);
}

void launch_pad64(int n, int kd, int dir, double* Z, double* P, hipStream_t st) {
    const long long tot = (long long)n * kd;
    if (tot) k_pad64<<<(int)((tot + 255) / 256), 256, 0, st>>>(n, kd, dir, Z, P);
}

}  // namespace feti
