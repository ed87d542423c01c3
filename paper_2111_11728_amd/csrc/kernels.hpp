// Host-side launchers of the FETI kernels and the device views they take.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <vector>
#include <cstdint>

#include "common.hpp"

namespace feti {

// F*Lambda work item: one workgroup per tile, all rows of one subdomain's augmented operator
// A_s = [F_s; F_rc^sT] in 16-row blocks: n_red blocks from red0 in the reduced precision (two
// per wavefront) and n_d blocks from d0 in FP64 (one per wavefront; with an odd n_red the last
// reduced wavefront also takes block d0): (n_red+1)/2 + n_d - (n_red odd && n_d > 0) <= 16.
// kFlSplitK tiles hold n_d <= 4 FP64 blocks with the contraction split four ways.
constexpr int kFlWaves = 16;   // wavefronts per F*Lambda workgroup
struct FlTile {
    int s, red0, n_red, d0, n_d, flags, pad1, pad2;   // s < 0: empty slot
};
constexpr int kFlNoT = 1;     // FlTile flag: reduced row blocks do not write the F_rc^T rows
constexpr int kFlSplitK = 2;  // FlTile flag: one FP64 row block, contraction split over all wavefronts
struct FlTiles {
    const FlTile* t = nullptr;
    int n = 0;
};

// Descriptors of batched dense operations (offsets in elements from a base pointer).
struct GemmDesc {   // C[m x n] = beta C + alpha A^T B, A: k x m (lda), B: k x n (ldb), row-major
    long long a, b, c;
    int m, n, k, lda, ldb, ldc;
};
struct PotrfDesc {
    long long a;
    int n, lda;
};
struct TrsmDesc {   // B <- L^{-1} B, L: n x n (ldl), B: n x ncols (ldb), row-major
    long long l, b;
    int n, ldl, ncols, ldb;
};

// first Gram workgroup of each design of a segmented product (w[nseg] = total), by value
constexpr int kMaxSegDesigns = 64;
struct SegBases {
    int w[kMaxSegDesigns + 1];
};
// FETI-DP coarse matrix Kbar_cc of several independent designs is block diagonal: one dense
// block per design (corners cg0 .. cg0 + n - 1, row-major at off in the block buffer).
struct CoarseBlk {
    int cg0, n;
    long long off;
};
struct CoarseTile {   // 16 rows r0 .. r0 + 15 (block-local) of block blk
    int blk, r0;
};
// One design's rows in a segmented Krylov block (several designs, each with its own search
// directions in the same 64 columns): rows row0 .. row0 + nrows - 1 (nrows a multiple of 256;
// every 256-row block belongs to one design), base = its share of the Gram workgroups.
struct KrySeg {
    int row0, nrows, base;
};

// Host-side launch parameters of one design inside a context holding several (a single design
// has one entry with zero offsets).
struct DesignDev {
    int sub0 = 0, lam0 = 0, n_lambda = 0;
    long long el0 = 0, n_el = 0, dof0 = 0, n_dof = 0;
    int nel[3] = {1, 1, 1}, nsub[3] = {1, 1, 1};
    const int* axf[3] = {nullptr, nullptr, nullptr};
    const int* axc[3] = {nullptr, nullptr, nullptr};
};

// Device copies of the topology (pointers into one device allocation).
struct DevTopo {
    int dim = 2, n_sub = 0, n_lambda = 0, n_cg = 0, n_groups = 0, n_rbm = 0;
    int nel[3] = {0, 0, 0}, nsub[3] = {1, 1, 1};
    int max_nodes = 0, max_beta = 0, max_nb = 0, max_rows_F = 0, max_nloc = 0, max_nc = 0, max_ni = 0;
    int max_line = 0, max_planes = 0;   // DOFs of the longest line; lines (planes) per subdomain
    // coarse blocks (one per design) and the 16-row tiles of the coarse solve
    const int* cg_blk = nullptr;
    const CoarseBlk* cblk = nullptr;
    const CoarseTile* ctiles = nullptr;
    int n_ctiles = 0;
    std::vector<DesignDev> dsg;   // host side: per-design ranges for the per-design launches
    const int* seg = nullptr;     // device: (first lambda row, rows) per design
    // segmented Krylov (several designs with their own directions): per-design row ranges and
    // the design of every 256-row block; null / empty for one design
    const KrySeg* kseg = nullptr;
    std::vector<KrySeg> hkseg;
    const int* rb_design = nullptr;
    const double* K0dev = nullptr;    // unit-modulus element matrix (row-major)
    long long nb_tot = 0, nc_tot = 0, ni_tot = 0, nloc_tot = 0, n_dof = 0;
    const SubMeta* subs = nullptr;
    const LineMeta* lines = nullptr;
    const int8_t* lcls = nullptr;
    const int* lidx = nullptr;
    const int* lglob = nullptr;
    const int8_t* lown = nullptr;
    const int* i_loc = nullptr;
    const int* b_loc = nullptr;
    const int* c_loc = nullptr;
    const int* c_glob = nullptr;
    const int* bq_s = nullptr;       // subdomain of every b DOF
    const int* row_s = nullptr;
    const int* row_j = nullptr;
    const int8_t* row_sg = nullptr;
    const long long* row_yo = nullptr;   // [2 n_lambda]: off_b + row_j of each side (-1: none)
    const int* row_sh = nullptr;
    const int* sh_ptr = nullptr;
    const int* sh_s = nullptr;
    const int* sh_l = nullptr;
    const int* bg_ptr = nullptr;
    const int* bg_row = nullptr;
    const int8_t* bg_sg = nullptr;
    const int* cc_ptr = nullptr;
    const int* cc_s = nullptr;
    const int* cc_j = nullptr;
    const int* ax_first[3] = {nullptr, nullptr, nullptr};
    const int* ax_cnt[3] = {nullptr, nullptr, nullptr};
    const int4* ps_work = nullptr;    // preconditioner workgroups: (subdomain, part g, parts G_s, 0)
    const int* ps_G = nullptr;        // parts G_s of every subdomain
    int ps_nwg = 0, ps_maxG = 1;
    const int* gmap = nullptr;        // fixed-width gather map: gmap[q*gmap_R + t] = sign*(row+1), 0 unused
    int gmap_R = 1;
    // FETI-DP coarse fold of every lambda row, fixed width fr_w: the row's entries of
    // B_r F_rc B_c (n_lambda x n_cg, at most two subdomains' corners), sign included
    const int* fr_n = nullptr;        // entries of each row
    const int* fr_col = nullptr;      // [n_lambda x fr_w] global corner DOF
    double* fr_val = nullptr;         // [n_lambda x fr_w] values (set up with F_rc)
    int fr_w = 0;
    // the same rows grouped by their pair of subdomains (n_pairs = 0: not built): the rows at
    // positions pr_ptr[g] .. pr_ptr[g+1]), the union of their corner DOFs pu_cg[pu_ptr[g] .. ),
    // and the position of every fold entry in its group's union
    int n_pairs = 0;
    const int* pr_ptr = nullptr;
    const int* pu_ptr = nullptr;
    const int* pu_cg = nullptr;
    const int* fr_pos = nullptr;      // [pair position x fr_w], in the group order
    // per row in the group order: pr_rec = {side 0's local product row off_b + j (or -1), the
    // same for side 1, fold entry count << 2 | (sign_0 < 0) | (sign_1 < 0) << 1, lambda row};
    // the fold values; pr_ipos[row] = the row's position
    const int4* pr_rec = nullptr;
    double* pr_fval = nullptr;
    const int* pr_ipos = nullptr;
    int n_lines_tot = 0;              // interior line (2D) / plane (3D) blocks over all subdomains
    FlTiles fl64;                     // F*Lambda work list with every row block in FP64
    FlTiles flred;                    // ... with every row block in the reduced precision
};

// ---- setup (k_setup.hip) ----
// rows of K^s coupling interior and interface DOFs, applied from the element densities:
// to_beta = 0: out_i = f_i - K_i,beta in_beta; to_beta = 1: out_beta = f_beta - K_beta,i in_i
void launch_coupling(const DevTopo& t, const double* Emod, int to_beta, const double* in, const double* f, double* out,
                     hipStream_t st);
// Emod[e] = Emin + rho_e^p (E0 - Emin), e < n
void launch_simp_moduli(long long n, const double* rho, double p, double E0, double Emin, double* Emod,
                        hipStream_t st);
void launch_assemble(const DevTopo& t, const double* Emod, double* L, double* Z, double* S, double* diag,
                     hipStream_t st);
// Block-tridiagonal Cholesky, plane by plane batched over the subdomains; ws holds
// bt_plane_ws_bytes(t) bytes (per-plane Cholesky descriptors and pivot flags)
size_t bt_plane_ws_bytes(const DevTopo& t);
void launch_bt_factor(const DevTopo& t, double* L, int* info, void* ws, hipStream_t st);
// Block-tridiagonal Cholesky that also writes L_kk^{-1} (lines <= 128 DOFs; otherwise the
// plane-by-plane factorisation, and launch_bt_invert must follow)
void launch_bt_factor_li(const DevTopo& t, double* L, double* Li, int* info, void* ws, hipStream_t st);
// Z <- L^{-1} Z with the explicit diagonal inverses (matrix cores; lines <= 128 DOFs)
void launch_bt_forward_li(const DevTopo& t, const double* L, const double* Li, double* Z, hipStream_t st);
void launch_bt_forward(const DevTopo& t, const double* L, double* Z, hipStream_t st);
// Z <- L^{-1} Z plane by plane with the explicit inverses (matrix cores, batched over the
// subdomains; lines of more than kSweepMaxLine and at most kSweepBigLine DOFs); T: work buffer of
// bt_plane_fwd_doubles(t) doubles
long long bt_plane_fwd_doubles(const DevTopo& t);
void launch_bt_forward_planes(const DevTopo& t, const double* L, const double* Li, double* Z, double* T,
                              hipStream_t st);
// along one dimension of C over the batch
// Deflation of local interface modes: subspace width, the largest interface block held in LDS,
// modes per subdomain, subspace iterations and the relative spectral gap that ends a selection
constexpr int kDeflSubspace = 16;
constexpr int kDeflMaxNb = 576;
constexpr int kDeflMaxModes = 8;
constexpr int kDeflIters = 40;
constexpr double kDeflGap = 0.05;
// omega (summed weights of each interface DOF), DL = F_s, DM = omega S~ omega (n_b x n_b at off_P)
void launch_defl_local(const DevTopo& t, const double* F64, const double* Pk, const double* bg_w, double* omega,
                       double* DL, double* DM, hipStream_t st);
void launch_defl_tril(const DevTopo& t, double* DL, hipStream_t st);
void launch_defl_eig(const DevTopo& t, const double* DC, const double* DB, const double* omega, int m, double tau,
                     double gap, int n_it, double* U, double* mu, int* cnt, hipStream_t st);
void launch_defl_scatter(const DevTopo& t, const double* bg_w, const double* U, const int* col0, const int* cnt,
                         double* Y, hipStream_t st);
// the first kd columns of the n x 64 block P from the n x kd block Z (dir 0), or back (dir 1)
void launch_pad64(int n, int kd, int dir, double* Z, double* P, hipStream_t st);
// C = beta C + alpha A^T B per matrix of the batch; tdim: the largest number of 64-wide tiles
// along one dimension of C over the batch
void launch_gemm_tn(const GemmDesc* d, int nbatch, int tdim, const double* A, const double* B, double* C,
                    double alpha, double beta, int symmetric, hipStream_t st);
// max_n: the largest n of the batch (above 512 the blocked multi-workgroup form runs)
void launch_potrf(const PotrfDesc* d, int nbatch, int max_n, double* base, int* info, hipStream_t st);
// B <- L^{-1} B with B the identity on entry (B = L^{-1} on exit)
void launch_trsm_identity(const TrsmDesc* d, int nbatch, int max_cols, const double* L, double* B, hipStream_t st);
void launch_copy_Sbb(const DevTopo& t, const double* S, double* dst, int identity, hipStream_t st);
void launch_tfeti_rbm(const DevTopo& t, const double* S, double* Rb, double* Cit, double* tau, double* W,
                      hipStream_t st);
void launch_tfeti_fix(const DevTopo& t, const double* Rb, const double* tau, double* F64, hipStream_t st);
void launch_frc(const DevTopo& t, const double* S, double* F64, double* Kc, hipStream_t st);
void launch_swizzle(const DevTopo& t, const double* F64, double* sw64, float* sw32, __hip_bfloat16* hi,
                    __hip_bfloat16* lo, hipStream_t st);
void launch_weights(const DevTopo& t, int kscale, const double* diag, double* w, double* bg_w, hipStream_t st);
void launch_coarse_assemble(const DevTopo& t, const double* Kc, double* Kg, hipStream_t st);
void launch_ggt_assemble(const DevTopo& t, const double* Rb, double* GG, hipStream_t st);
void launch_set_identity(double* A, int n, long long lda, hipStream_t st);

// ---- operator application (k_apply.hip) ----
// Y/T outputs of the local products: Y [nb_tot x k], T [nc_tot x k], row-major, type by precision.
// Ared/Ared_lo: swizzled A_s in the reduced precision (BF16X3: hi and lo parts), A64: in FP64.
// tl = nullptr: every row block in `precision`; out_f64: write Y/T in FP64 whatever the precision
void launch_flambda(const DevTopo& t, int precision, int k, const double* Lambda, const void* Ared,
                    const void* Ared_lo, const double* A64, void* Y, void* T, hipStream_t st,
                    const FlTiles* tl = nullptr, int out_f64 = 0);
// Copy F_s (leading n_b x n_b block of the augmented operator) into dst (ld n_b), rounded to
// the given precision (FP64: exact; FP32; BF16X3: hi + lo split) and back to FP64.
void launch_copy_F_rounded(const DevTopo& t, const double* F64, int precision, double* dst, hipStream_t st);
// dev[s] = max_j |L2_jj^2 / L1_jj^2 - 1| over the Cholesky factors L1 (exact) and L2 (rounded)
// stored in W1 / W2 (infinite if info2[s] != 0)
void launch_pivot_compare(const DevTopo& t, const double* W1, const double* W2, const int* info2, double* dev,
                          hipStream_t st);
// t = add + sum_s B_c^sT T_s (n_cg x k, in tbuf), v = scale * Kinv t
void launch_coarse(const DevTopo& t, int k, int ytype_f32, const void* T, const double* add, const double* Kinv,
                   double scale, double* v, double* tbuf, hipStream_t st);
// Y_s += F_rc^s v_s (coarse correction folded into the local products)
void launch_fold_coarse(const DevTopo& t, int k, int ytype_f32, const double* F64, const double* v, void* Y,
                        hipStream_t st);
// Q[row] = sum over sides sign * Y[b]
void launch_scatter(const DevTopo& t, int k, int ytype_f32, const void* Y, double* Q, hipStream_t st);
// module types: per-subdomain density hashes, element-wise comparison of (member, representative)
// pairs, and rows gathered by a map (per-subdomain setup results of representatives)
void launch_rho_hash(const DevTopo& t, const double* rho, unsigned long long* out, hipStream_t st);
void launch_rho_match(const DevTopo& t, const double* rho, const int* pairs, int npairs, int* flag, hipStream_t st);
void launch_gather_rows(int n, int w, const int* map, const double* src, double* dst, hipStream_t st);
constexpr int kFoldPairMaxU = 64;   // corner DOFs of two subdomains staged per group
constexpr int kFoldRows = 4;        // rows per wavefront and pass of the pair scatter-fold
constexpr int kFoldPairMaxW = 32;   // widest fold row (entries) taken by the pair scatter-fold
constexpr int kFoldPairMinRows = 96;   // shortest mean group (rows) taken by the pair scatter-fold
// fr_val from the F_rc^T rows of the augmented operators (after launch_frc)
void launch_fold_rows(const DevTopo& t, const double* F64, hipStream_t st);
// Q = sum_s B_s Y_s + (B_r F_rc B_c) v: the scatter with the coarse fold of F*Lambda in one pass
void launch_scatter_fold(const DevTopo& t, int k, int ytype_f32, const void* Y, const double* v, double* Q,
                         hipStream_t st);
// x_s = B~^sT r gathered and multiplied: y_s = P_s x_s, P_s symmetric in packed 64x64 upper tiles;
// ypart: kPsMaxSplit * nb_tot doubles of workspace (subdomains split over several workgroups)
constexpr int kPsMaxSplit = 8;
// super-lumped preconditioner: y = diag(K_bb) B~^T r per interface DOF; Pk reduced to its diagonal
void launch_precond_diag(const DevTopo& t, const double* r, const double* bg_w, const double* Pk, double* y,
                         hipStream_t st);
void launch_pk_diag_only(const DevTopo& t, double* Pk, hipStream_t st);
void launch_precond_local(const DevTopo& t, const double* r, const double* bg_w, const double* Pk, double* ypart,
                          double* y, hipStream_t st);
// the same from FP32 copies of the packed tiles (FP64 products and sums)
void launch_precond_local32(const DevTopo& t, const double* r, const double* bg_w, const float* Pk32,
                            double* ypart, double* y, hipStream_t st);
// b[i] = a[i] rounded to FP32, i < n
void launch_round_f32(long long n, const double* a, float* b, hipStream_t st);
// Pk (packed upper tiles) <- the leading n_b x n_b block of S (ld n_beta)
void launch_pack_sym(const DevTopo& t, const double* S, double* Pk, hipStream_t st);
// Z[row][g(s)] = sum over sides sign * w * y_s[j]; one_column sums into column 0
void launch_precond_scatter(const DevTopo& t, int one_column, const double* w, const double* y, double* Z,
                            hipStream_t st);
// TFETI projector pieces
void launch_proj_G(const DevTopo& t, int k, const double* Y, const double* Rb, double* GY, hipStream_t st);
void launch_small_gemm(int m, int n, int kk, const double* A, const double* B, double* C, double alpha,
                       hipStream_t st);  // C[m x n] = alpha A[m x kk] B[kk x n], row-major, B/C ld n
void launch_proj_apply(const DevTopo& t, int k, const double* tcoef, const double* Rb, double sign, double* Y,
                       hipStream_t st);  // Y[row] += sign * sum_sides sg * Rb[j] . tcoef[s]

// ---- Krylov (k_krylov.hip) ----
// partial Gram: for every block b < nblk (A_b = Aptrs[b]) and row chunk c:
// part[(b*nchunk + c)][ka x kb] = A_b[rows of c]^T B[rows of c]. f32 (ka = kb = 64 only): the
// products on the FP32 matrix cores from the FP64 operands rounded in registers, FP32 partial sums
// over each wavefront's rows, FP64 beyond.
void launch_gram(int n, int ka, int kb, const double* const* Aptrs, int nblk, const double* B, double* part,
                 double* out, hipStream_t st, bool f32 = false);
int gram_chunks(int n, int nblk);
constexpr long long kGramPartCap = 4 * 4096ll * kMaxDirs * kMaxDirs;   // doubles in the partial-sum buffer
// out = beta C + alpha sum_b A_b M_b (FP64 matrix cores; f32 with kd = 64: the sum on the FP32
// matrix cores, the update in FP64), A_b n x kd, M_b kd x kd
// Segmented forms (kd = 64, several designs): Gram products per design (out[(d*nblk + b)*4096]),
// products whose 64x64 matrix is the row's design's (Mats + design * mstride), gamma per design,
// lambda/r update with each row's design's gamma, one pivoted Cholesky per design, rows of
// frozen designs zeroed.
void launch_gram_seg(const DevTopo& t, int n, const double* const* Aptrs, int nblk, const double* B, double* part,
                     double* out, hipStream_t st, bool f32 = false);
void launch_ts_seg(const DevTopo& t, int n, int nblk, const double* const* Aptrs, const double* Mats, long long mstride,
                   const double* C, double* out, double alpha, double beta, hipStream_t st, bool f32 = false);
void launch_ts_pair_seg(const DevTopo& t, int n, const double* const* Aptrs, const double* const* Aptrs2,
                        const double* Mats, double* out, double* out2, hipStream_t st);
void launch_gemv_t_seg(const DevTopo& t, int n, const double* A, const double* x, double* part, double* out,
                       hipStream_t st);
void launch_update_lr_seg(const DevTopo& t, int n, const double* W, const double* Q, const double* g, double* lam,
                          double* r, hipStream_t st);
void launch_pivchol_seg(int nseg, const double* D, double rr_tol, double* T, int* rank, unsigned long long* kept_mask,
                        hipStream_t st);
void launch_zero_rows(const DevTopo& t, int n, unsigned long long frozen, double* Z, hipStream_t st);
// out = A Mats and out2 = A2 Mats (one stored block each, n x kd; Mats kd x kd) in one launch
void launch_ts_pair(int n, int kd, const double* const* Aptrs, const double* const* Aptrs2, const double* Mats,
                    double* out, double* out2, hipStream_t st);
void launch_ts_gemm(int n, int kd, int nblk, const double* const* Aptrs, const double* Mats, const double* C,
                    double* out, double alpha, double beta, hipStream_t st, bool f32 = false);
// the n scalars src, then seq, into the host-mapped dst (seq last, after a system-scope fence)
void launch_publish(const double* src, int n, double* dst, long long seq, hipStream_t st);
void launch_pivchol(int k, const double* D, double rr_tol, double* T, int* rank, hipStream_t st,
                    unsigned long long* kept_mask = nullptr);   // kept_mask: bit j set when column j was kept
// Z[:, c] = 0 for the columns c set in mask (n x k row-major)
void launch_zero_cols(long long n, int k, unsigned long long mask, double* Z, hipStream_t st);
void launch_apply_T(int n, int k, const double* T, const double* W, const double* Q, double* Wo, double* Qo,
                    hipStream_t st);
// SIMP optimality-criteria step: partial volumes sum rho_e(L) (mode 0) or maxima of |dc| (mode 1)
// per workgroup into part[nwg]; then rho_new = rho(L)
void launch_oc_reduce(long long n, const double* rho, const double* dc, double lam, double move, double eta,
                      double rho_min, int mode, int nwg, double* part, hipStream_t st);
void launch_oc_apply(long long n, const double* rho, const double* dc, double lam, double move, double eta,
                     double rho_min, double* out, hipStream_t st);
// lam += W g; r -= Qg_scale * Q g  (Q may be null)
// lam_out = lam + W g (lam_out = nullptr: in place), r -= Q g (Q = nullptr: r untouched)
void launch_update_lr(int n, int k, const double* W, const double* Q, const double* g, double* lam, double* r,
                      hipStream_t st, double* lam_out = nullptr);
void launch_orth_update(int n, int k, const double* const* Wptrs, int nblk, const double* Psi, double* W,
                        hipStream_t st);
void launch_rowsum_dot(int n, int k, const double* r, const double* Z, double* part, double* out, hipStream_t st);
// out[d] = sum over the lambda rows of design d of r[row] * sum_c Z[row][c] (k columns), fixed order
void launch_seg_dot(const DevTopo& t, int k, const double* r, const double* Z, double* part, double* out,
                    hipStream_t st);   // part: scratch of 8 doubles per design
// out[0..63] = A^T x (A: n x 64 row-major), two-stage deterministic reduction through part
void launch_gemv_t(int n, int k, const double* A, const double* x, double* part, double* out, hipStream_t st);
void launch_diff_norms(long long len, const double* a, const double* b, double* part, double* out,
                       hipStream_t st);  // out[0] = ||a - b||^2, out[1] = ||b||^2 (part: >= 512)
void launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t st);  // y = a x + b y
void launch_pcg_update(int n, const double* sc, const double* w, const double* q, double* lam, double* r,
                       hipStream_t st);
void launch_pcg_dir(int n, const double* sc, const double* z, double* w, hipStream_t st);

// ---- solve-phase (k_solve.hip) ----
void launch_scatter_f(const DevTopo& t, const double* f, double* fi, double* fbeta, hipStream_t st);
// Li: explicit inverses of the diagonal Cholesky blocks (LineMeta::off_inv), used when every
// line has at most kSweepMaxLine DOFs
void launch_bt_fsolve1(const DevTopo& t, const double* L, const double* Li, double* h, hipStream_t st);
void launch_bt_bsolve1(const DevTopo& t, const double* L, const double* Li, double* x, hipStream_t st);
void launch_bt_invert(const DevTopo& t, const double* L, double* Li, hipStream_t st);
constexpr int kSweepMaxLine = 128;
// longest line that still gets explicit diagonal inverses (launch_bt_invert) and the tiled sweeps
constexpr int kSweepBigLine = 512;
// g = fbeta - Z^T h; part: scratch of 8 (nb_tot + nc_tot) doubles
void launch_zt_gemv(const DevTopo& t, const double* Z, const double* h, const double* fbeta, double* g, double* part,
                    hipStream_t st);
void launch_z_gemv(const DevTopo& t, const double* Z, const double* ubeta, const double* h, double* x,
                   hipStream_t st);   // x = h - Z ubeta
void launch_local_F(const DevTopo& t, const double* F64, const double* g, double* yb, double* yc, hipStream_t st);
void launch_fbar(const DevTopo& t, const double* g, const double* yc, double* fbar_s, hipStream_t st);
void launch_gather_B(const DevTopo& t, const double* lam, double* xb, hipStream_t st);   // xb = B^T lam per subdomain
// scratch: nb_tot doubles
void launch_dp_ub(const DevTopo& t, const double* F64, const double* S, const double* g, const double* xb,
                  const double* uc, double* ubeta, double* scratch, hipStream_t st);
void launch_tfeti_ub(const DevTopo& t, const double* F64, const double* g, const double* xb, double* ubeta,
                     double* scratch, hipStream_t st);
void launch_tfeti_e(const DevTopo& t, const double* fi, const double* fbeta, const double* Cit, double* e,
                    hipStream_t st);
void launch_assemble_loc(const DevTopo& t, const double* ui, const double* ubeta, const double* Cit,
                         const double* alpha, double* uloc, hipStream_t st);
void launch_average(const DevTopo& t, const double* uloc, double* u, hipStream_t st);
void launch_compliance(const DevTopo& t, const double* f, const double* u, const double* rho, double p, double E0,
                       double Emin, double* part, double* c, double* g, hipStream_t st);

}  // namespace feti
