// Shared device-side definitions of the FETI library (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>

#include "classes.hpp"
#include "feti.h"

namespace feti {

constexpr int kMaxDirs = 64;      // widest block of search directions per launch
constexpr int kWG = 256;          // threads per workgroup of the setup kernels (4 wavefronts)

// Per-subdomain metadata, one struct per subdomain in device memory.
struct SubMeta {
    int lo[3];          // first element per axis
    int nn[3];          // local nodes per axis
    int n_loc, n_i, n_b, n_c, n_beta, grp;
    int n_lines;        // block-tridiagonal blocks of K_ii (grid rows in 2D, planes in 3D)
    int ldF;            // leading dimension (columns) of the row-major F_s storage, n_b rounded up to 16
    int rows_F;         // rows of the augmented operator [F_s; F_rc^T]: n_b + n_c rounded up to 16
    int rowT;           // first row of F_rc^T (= n_b: the corner rows follow F_s directly)
    int nelx, nely;     // element grid of the subdomain's design (its global element numbering)
    long long el0;      // first element of the subdomain's design in the density array
    long long off_loc, off_i, off_b, off_c;   // prefix offsets of the per-DOF arrays
    long long line0;    // first entry of this subdomain in the line table
    long long off_L;    // block-tridiagonal factor storage (doubles)
    long long off_Z;    // Z = L^{-1} K_i,beta, row-major [n_i x n_beta]
    long long off_S;    // S = K_beta,beta - Z^T Z, row-major [n_beta x n_beta]
    long long off_F;    // [rows_F x ldF] row-major F_s and F_rc^T (FP64 master copy)
    long long off_Fsw;  // MFMA-swizzled copies (elements, same offset for every precision)
    long long off_P;    // work buffers of n_b x n_b, row-major
    long long off_Pk;   // preconditioner block S~: upper triangle in 64x64 tiles (I <= J), tile (I, J) at
                        // (J(J+1)/2 + I) * 4096, holding S~[64I + a][64J + b] at a*64 + b (zero past n_b)
    long long off_Kc;   // Kbar_cc^s [n_c x n_c]
    long long off_R;    // TFETI: R_b [n_b x n_rbm] row-major
};

// One block (grid line / plane) of the block-tridiagonal interior matrix.
struct LineMeta {
    int i0;             // first interior index of the block
    int n;              // interior DOFs in the block
    int n_prev;         // interior DOFs of the previous block (0 for the first)
    int pad_;
    long long off_diag; // n x n dense diagonal block (lower triangle holds L_kk after factorisation)
    long long off_sub;  // n x n_prev dense block coupling to the previous block (L_{k,k-1})
    long long off_inv;  // n x n explicit L_kk^{-1} (lower triangle) in the inverse buffer
};

__device__ __forceinline__ double warp_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// v of the lane CTRL selects within its row of 16 (a DPP move of both halves of a double)
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    const int nlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
    const int nhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)nhi << 32) | (unsigned int)nlo);
}

// sum over the lane's row of 16 lanes, left in every lane of the row (DPP: xor 1, xor 2,
// rotate 4, rotate 8; every lane of the row must be active)
__device__ __forceinline__ double row16_sum_dpp(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x124>(v);   // row_ror:4
    v += dpp_mov<0x128>(v);   // row_ror:8
    return v;
}

// sum over a full wavefront without LDS: DPP within rows of 16 (xor 1, xor 2, rotate 4,
// rotate 8 leave every lane with its row's sum), then the four row sums through readlane in a
// fixed order (uniform result; every lane must be active)
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v = row16_sum_dpp(v);
    auto rl = [&](int lane) {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    };
    return (rl(0) + rl(16)) + (rl(32) + rl(48));
}

typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef double v4d_t __attribute__((ext_vector_type(4)));

// Streamed operands go through buffer resources covering exactly the rows a wavefront owns:
// a load past num_records returns zeros without touching memory, so the loads of the ring
// are unconditional (no per-lane branches, no zero fill) and the compiler can count them.
typedef unsigned v4u_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const double* base, int nbytes) {
    // wavefront-uniform by construction; readfirstlane keeps the descriptor in scalar registers
    // (a per-lane copy would turn every load into a loop over distinct descriptors)
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0,
                                             __builtin_amdgcn_readfirstlane(nbytes), 0x00020000);
}
__device__ __forceinline__ v4d_t load4d(__amdgpu_buffer_rsrc_t r, int off) {
    const v2d_t lo = __builtin_bit_cast(v2d_t, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    const v2d_t hi = __builtin_bit_cast(v2d_t, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0));
    return v4d_t{lo[0], lo[1], hi[0], hi[1]};
}

}  // namespace feti
