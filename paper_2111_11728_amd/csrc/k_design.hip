// SIMP design update (Sec. 1: minimum compliance under a bound on the material volume, with the
// modulus law of Eq. 1): one optimality-criteria step per call.
//   B_e(L)   = max(0, -dc_e) / L
//   rho_e(L) = min(min(1, rho_e + move), max(max(rho_min, rho_e - move), rho_e B_e(L)^eta))
// The volume sum_e rho_e(L) is non-increasing in L; the host brackets and bisects L on the
// per-workgroup partial volumes these kernels return (summed on the host in a fixed order, so
// every decision is reproducible), then writes rho(L).
#include "kernels.hpp"

namespace feti {

__device__ __forceinline__ double oc_value(double rho, double dc, double lam, double move, double eta, double rho_min) {
    const double b = fmax(0.0, -dc) / lam;
    const double cand = rho * pow(b, eta);
    const double lo = fmax(rho_min, rho - move), hi = fmin(1.0, rho + move);
    return fmin(hi, fmax(lo, cand));
}

// part[blockIdx.x] = sum over the workgroup's elements of rho_e(L) (mode 0) or of |dc_e| as a
// maximum (mode 1); each thread walks a fixed grid-stride sequence, the workgroup then sums its
// 256 values in a fixed order (DPP rows, then the four wavefront sums through LDS)
__global__ void __launch_bounds__(256) k_oc_reduce(long long n, const double* __restrict__ rho,
                                                   const double* __restrict__ dc, double lam, double move, double eta,
                                                   double rho_min, int mode, double* __restrict__ part) {
    __shared__ double ws[4];
    double acc = 0.0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += 256LL * gridDim.x) {
        if (mode == 0)
            acc += oc_value(rho[e], dc[e], lam, move, eta, rho_min);
        else
            acc = fmax(acc, fabs(dc[e]));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (mode == 0) {
        acc = wave_sum_dpp(acc);
    } else {
        for (int o = 32; o > 0; o >>= 1) acc = fmax(acc, __shfl_xor(acc, o, 64));
    }
    if (lane == 0) ws[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        part[blockIdx.x] = mode == 0 ? (ws[0] + ws[1]) + (ws[2] + ws[3]) : fmax(fmax(ws[0], ws[1]), fmax(ws[2], ws[3]));
}

__global__ void __launch_bounds__(256) k_oc_apply(long long n, const double* __restrict__ rho,
                                                  const double* __restrict__ dc, double lam, double move, double eta,
                                                  double rho_min, double* __restrict__ out) {
    const long long e = blockIdx.x * 256LL + threadIdx.x;
    if (e < n) out[e] = oc_value(rho[e], dc[e], lam, move, eta, rho_min);
}

void launch_oc_reduce(long long n, const double* rho, const double* dc, double lam, double move, double eta,
                      double rho_min, int mode, int nwg, double* part, hipStream_t st) {
    if (n > 0) k_oc_reduce<<<nwg, 256, 0, st>>>(n, rho, dc, lam, move, eta, rho_min, mode, part);
}

void launch_oc_apply(long long n, const double* rho, const double* dc, double lam, double move, double eta,
                     double rho_min, double* out, hipStream_t st) {
    if (n > 0) k_oc_apply<<<(int)((n + 255) / 256), 256, 0, st>>>(n, rho, dc, lam, move, eta, rho_min, out);
}

}  // namespace feti
