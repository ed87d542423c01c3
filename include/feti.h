/*
 * feti.h - C ABI of the MI355X FETI library (Total FETI and FETI-DP with k-scaling,
 * full orthogonalisation and rank-revealing simultaneous search directions) for
 * SIMP-heterogeneous linear elasticity on structured Q4 / Hex8 grids.
 *
 * Method: Medricky, Doskar, Pultarova, Zeman, "Comparison of FETI-based domain
 * decomposition methods for topology optimization problems", arXiv 2111.11728.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Grid: unit square (cube) elements, thickness 1. Nodes are numbered
 *   lexicographically, x fastest; DOFs are interleaved, dof = dim*node + component;
 *   elements are numbered lexicographically, x fastest.
 * - Subdomains are the boxes of a tensor-product partition, numbered x fastest.
 *   Local DOFs of a subdomain follow the same lexicographic rule inside its box.
 * - Lagrange-multiplier rows (lambda) are ordered node by node in increasing global
 *   node number, then component, then Dirichlet rows by subdomain (TFETI only) or
 *   gluing pairs (a, b), a < b, with +1 on a and -1 on b. Every free DOF shared by m
 *   subdomains gets all m(m-1)/2 pairs (redundant at cross-points, Sec. 3.1).
 * - Blocks of lambda vectors are row-major [n_lambda x k] (k contiguous).
 * - Unless stated otherwise every array argument is a DEVICE pointer, read or
 *   written in stream order on the stream given to feti_setup; the caller owns it
 *   and the library keeps no reference to it after the call returns. Host
 *   pointers are marked "host".
 * - No entry point throws; each returns a feti_status. On error the message is
 *   available from feti_last_error() (thread-local) and outputs are unspecified,
 *   except FETI_ENOCONV / FETI_EBREAKDOWN from feti_solve, which still write u and info.
 */
#ifndef FETI_H
#define FETI_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct feti_ctx feti_ctx;

typedef enum {
    FETI_OK = 0,
    FETI_EINVAL = -1,      /* invalid argument (sizes, densities, options) */
    FETI_ENOMEM = -2,      /* device or host allocation failed */
    FETI_EHIP = -3,        /* a HIP runtime call or kernel launch failed */
    FETI_ENOTSPD = -4,     /* non-positive pivot in a subdomain or coarse Cholesky */
    FETI_ENOCONV = -5,     /* max_it reached before the tolerance; u and info written */
    FETI_EBREAKDOWN = -6   /* Krylov breakdown: no independent direction left (rank 0) */
} feti_status;

enum { FETI_TFETI = 0, FETI_DP = 1 };                       /* Sec. 2.1 / Sec. 2.2 */
enum { FETI_MULT = 0, FETI_KSCALE = 1 };                    /* Sec. 3.1 */
enum { FETI_PCG = 0, FETI_FO = 1, FETI_SFETI = 2 };         /* Sec. 2, Sec. 3.2, Sec. 3.3 */
enum { FETI_DIRICHLET = 0, FETI_LUMPED = 1, FETI_SUPERLUMPED = 2 };   /* Sec. 3.1, Eq. (13): S~^s =
                                                                       S^s, K_bb or diag K_bb */
enum { FETI_FP64 = 0, FETI_FP32 = 1, FETI_BF16X3 = 2 };     /* arithmetic of the F*Lambda product */
enum { FETI_PURE = 16 };          /* or-ed into feti_apply_F's precision: no per-subdomain FP64 fallback */
enum { FETI_PRECOND_FP32 = 2 };   /* or-ed into feti_apply_precond's one_column: FP32 blocks */

/* Structured grid and boundary conditions (Sec. 2, Eq. 2). */
typedef struct {
    int dim;                  /* 2 (bilinear Q4, plane stress) or 3 (trilinear Hex8) */
    int nel[3];               /* elements per axis (nel[2] ignored in 2D) */
    double nu;                /* Poisson ratio, in (-1, 0.5) */
    int n_fixed;              /* number of clamped global DOFs (value 0) */
    const int* fixed_dofs;    /* host: clamped global DOF numbers */
} feti_mesh;

/* Partition into subdomains (Sec. 2) and the grouping of subdomains into
 * simultaneous search directions (Sec. 3.3, Algorithm 1). */
typedef struct {
    int nsub[3];              /* subdomains per axis */
    const int* cuts[3];       /* host: per axis nsub[a]+1 increasing element indices from 0 to nel[a];
                                 NULL = uniform (nel[a] must then be divisible by nsub[a]) */
    int group[3];             /* S-FETI: subdomain blocks per axis forming one direction
                                 (0 or all 1 = one direction per subdomain) */
    int n_primal;             /* FETI-DP: nodes enforced in primal variables besides the corners
                                 (Sec. 2.2 Eq. 8-9 with the primal set enlarged as in Sec. 6, item i);
                                 0 = corners only */
    const int* primal_nodes;  /* host: n_primal global node numbers, each shared by two or more
                                 subdomains and carrying a free DOF (FETI_EINVAL otherwise); at
                                 most 32 primal DOFs per subdomain */
} feti_partition;

typedef struct {
    int method;               /* FETI_TFETI or FETI_DP */
    int scaling;              /* FETI_MULT or FETI_KSCALE */
    int krylov;               /* FETI_PCG, FETI_FO or FETI_SFETI */
    int precond;              /* FETI_DIRICHLET, FETI_LUMPED or FETI_SUPERLUMPED */
    int precision;            /* FETI_FP64, FETI_FP32 or FETI_BF16X3: arithmetic of F*Lambda inside
                                 the Krylov loop; Gram products, the coarse problem and the
                                 true residual stay FP64 */
    double tol;               /* stop when sqrt(r^T z) <= tol * sqrt(r_0^T z_0) (Eq. 16, relative) */
    int max_it;               /* Krylov iteration cap (<= 0: n_lambda) */
    double rr_tol;            /* rank-revealing pivot threshold on the Jacobi-scaled Gram matrix
                                 (<= 0: 1e-12) */
    int reorth;               /* passes of block classical Gram-Schmidt against the stored
                                 directions (1 or 2; 0 = 1, the single pass of Algorithm 1) */
    int max_refine;           /* mixed precision: FP64 residual restarts with the reduced-precision
                                 operator after the first pass (< 0: 4); further passes use FP64 */
    double relax;             /* mixed precision, switch level. > 0: an iteration applies the FP64
                                 operator while eps = sqrt(r^T z) > relax * eps0 and the reduced-
                                 precision one below it. <= 0 (default): measured switch. A reduced
                                 iteration moves the true residual away from the recursive one by
                                 about eta * eps, eta = ||(F_red - F) Z|| / ||F Z|| on the
                                 iteration's own block Z, so the reduced operator is used only while
                                 eta * eps <= 0.1 tol eps0. The first iteration that passes this test
                                 (with the prior eta = 1e-4 for FETI_FP32, 1e-3 for FETI_BF16X3),
                                 and every 16th reduced iteration after it, applies F in both
                                 precisions, keeps the FP64 product and records eta (the largest
                                 measurement is kept). */
    int graphs;               /* S-FETI: 1 = replay the per-iteration operator sequences (F*Lambda
                                 with the coarse correction, fold and scatter; the preconditioner
                                 with the residual dots) as captured hipGraphs, one per precision,
                                 recaptured after a setup or an autotune. Needs a non-null stream
                                 (capture is not allowed on the null stream); 0 = direct launches. */
    int orth_fp32;            /* S-FETI with 64 directions and a reduced precision, opt-in: 1 = an
                                 iteration on the reduced-precision operator also runs the block
                                 Gram-Schmidt against the stored directions on the FP32 matrix
                                 cores (FP64 history, FP64 update); probe iterations run both
                                 forms and keep the FP64 one. Its error is amplified by about
                                 sqrt(kappa(F)) in the F-inner product, so on strongly
                                 heterogeneous designs it stalls the reduced pass and the solve
                                 ends in FP64. 0 (default): FP64 on every iteration. */
    int warm_start;           /* 1 = a solve without lambda_init starts from the multipliers of the
                                 context's last solve, made feasible for the new load (lambda_0 +
                                 P lambda_prev; FETI-DP: lambda_prev), e.g. across the design
                                 iterations of a SIMP loop; its tolerance stays relative to the
                                 residual of the cold start lambda_0. Single design only; 0 = off */
    int recycle;              /* 1 = factorisation recycling over module types (Sec. 1; Sec. 2.1): at
                                 every setup, subdomains with the same local layout and bit-identical
                                 densities are found (a device hash per subdomain, then an element-by-
                                 element check) and only one of each group is factorised and gets its
                                 local operators, which the others then use. Results are bit-identical
                                 to a setup without recycling. Single design only; 0 = off */
    int defl_modes;           /* deflation of local interface modes (Sec. 6, item (ii): the
                                 interface modes that slow the iteration are found by local
                                 eigenproblems, as in GenEO, and taken out of the iteration).
                                 Reading: for every subdomain s, the eigenpairs of its local
                                 preconditioned operator P_s F_s (P_s its weighted preconditioner
                                 block on its dual rows, F_s its block of the dual operator),
                                 computed as C_s = L^T (omega S~ omega) L with F_s = L L^T and
                                 omega the summed weights of each interface DOF; of its largest
                                 eigenvalues, the k <= defl_modes (1..8) leading ones that end at
                                 a 5% spectral gap, mu_k >= 1.05 mu_{k+1}, and lie above defl_tau.
                                 The dual vectors y = diag(w_s) B_s S~ omega L x of all subdomains
                                 are made F-orthonormal once per setup; every solve corrects its
                                 start so that the residual is orthogonal to them, and FO, S-FETI
                                 and PCG orthogonalise each new search direction against them
                                 (deflated iterations). FETI-DP only, interface blocks of 32 to
                                 576 DOFs; 0 = off */
    double defl_tau;          /* deflation: smallest eigenvalue taken (0 = no threshold) */
    int precond_fp32;         /* FO or S-FETI with a reduced precision and the Dirichlet or lumped
                                 preconditioner: 1 = the passes on the reduced-precision operator
                                 apply the preconditioner (Sec. 3.1, Eq. 13) from an FP32 copy of its
                                 blocks, made at every setup, with FP64 products and sums. Its
                                 rounding changes only the search directions, which are then made
                                 F-orthogonal in FP64 against every stored direction; the dual
                                 iterate, the residual recurrence and the final FP64 true residual
                                 (tested with the FP64 preconditioner) are as before. Half the
                                 preconditioner's HBM reads. 0 (default) = FP64 blocks throughout;
                                 FETI_EINVAL for other combinations. */
} feti_opts;

typedef struct {
    int iters;                /* Krylov iterations over all passes */
    int refinements;          /* FP64 residual restarts performed */
    int status;               /* feti_status of the solve */
    double eps0;              /* sqrt(r_0^T z_0) */
    double eps;               /* final sqrt(r^T z) of the recurrence */
    double true_rel_res;      /* FP64 sqrt(r_t^T M r_t) / eps0 with r_t = P(d - F lambda) */
    int kept_directions;      /* total directions kept by the rank-revealing factorisation */
    double* res_hist;         /* host, optional: eps per iterate (first entry eps0) */
    int res_hist_cap;
    int* rank_hist;           /* host, optional: rank kept per iteration (same capacity) */
    double t_solve_ms;        /* wall time of feti_solve on the host clock */
    int fp64_fallback;        /* 1 if a reduced-precision pass broke down or stagnated and the
                                 solve was finished with the FP64 operator */
    int reduced_iters;        /* iterations that applied the reduced-precision operator */
    int precision_probes;     /* iterations that applied F in both precisions to measure eta */
    double reduced_rel_err;   /* largest eta measured (0 if never measured) */
    double reduced_orth_err;  /* orth_fp32: largest |Z_32 - Z_64| / |Z_64| of the orthogonalised
                                 block on probe iterations (0 if never measured) */
} feti_info;

typedef struct {
    int n_sub, n_dof, n_el, n_lambda, n_cg, n_alpha, n_groups;
    int nb_max, nb_min, n_loc_max, n_i_max, band_max;
    long long sum_nb2;        /* sum over subdomains of n_b^2 (entries of all explicit F_s) */
    long long sum_nb_nc;      /* sum over subdomains of n_b * n_c */
    long long device_bytes;   /* device memory held by a context */
    int n_fp64_subs;          /* FETI-DP with a reduced precision: subdomains whose F_s failed the
                                 round-off test at the last setup and run in FP64 */
    int n_designs;            /* independent designs held by the context (1 unless batched) */
    long long sum_nb2_fp64;   /* sum of n_b^2 over the subdomains counted by n_fp64_subs (their F_s
                                 products run on the FP64 matrix cores inside a reduced-precision solve) */
    int n_setup_subs;         /* subdomains factorised at the last setup (n_sub unless opts.recycle
                                 found repeated module types) */
    int n_defl;               /* opts.defl_modes: local modes selected at the last setup (all
                                 subdomains), and the F-orthonormal deflation directions kept */
    int n_defl_kept;
} feti_sizes;

/* One design of a batched context: its ranges in the concatenated arrays. */
typedef struct {
    long long el0, n_el;      /* densities and gradient: [el0, el0 + n_el) */
    long long dof0, n_dof;    /* loads and displacements: [dof0, dof0 + n_dof) */
    int sub0, n_sub;          /* subdomains */
    int lam0, n_lambda;       /* dual unknowns (rows of the multiplier vector) */
    int n_groups;             /* S-FETI direction groups of this design */
} feti_design;

/* Builds the integer topology only (no device work) and reports the interface sizes.
 * Host-only; usable without a GPU. */
feti_status feti_plan_sizes(const feti_mesh* mesh, const feti_partition* part,
                            const feti_opts* opts, feti_sizes* out);

/* Host-only: an adaptive choice of further FETI-DP primal nodes (Sec. 6, item i: compatibility
 * enforced in primal variables at nodes other than the corners), to pass in
 * feti_partition.primal_nodes. 2D: along every edge shared by two subdomains (its end vertices
 * excluded), a node's stiffness is the sum of the moduli Emin + rho_e^p (E0 - Emin) of its
 * elements (Sec. 1, Eq. 1), in lexicographic element order; the nodes whose stiffness is at least
 * theta times the edge's largest form runs of consecutive nodes, and the cap runs of largest total
 * stiffness (the earlier run on ties) each give their middle node ((first + last) / 2), unless it
 * carries no free DOF. 3D: no nodes. rho: host [n_el]. nodes: host, capacity nodes_cap, sorted
 * global node numbers (may be NULL to query the count in *n_out). cap <= 3 keeps a 2D subdomain
 * within the 32 primal DOFs of feti_partition. */
feti_status feti_adaptive_primal(const feti_mesh* mesh, const feti_partition* part, const double* rho, double p,
                                 double E0, double Emin, double theta, int cap, int* nodes, int nodes_cap,
                                 int* n_out);

/* Host-only export of the topology, for checking it against an independent
 * construction. what: 0 = per lambda row [side0 subdomain, side0 local DOF, side0 sign,
 * side1 subdomain (-1 if none), side1 local DOF, side1 sign] (6 ints per row);
 * 1 = per subdomain [n_loc, n_i, n_b, n_c, band] (5 ints); 2 = global corner DOFs.
 * out has capacity cap ints; *n_out receives the number written. */
feti_status feti_plan_export(const feti_mesh* mesh, const feti_partition* part,
                             const feti_opts* opts, int what, int* out, long long cap,
                             long long* n_out);

/* Setup (Sec. 2.1 / 2.2 operators, Sec. 3.1 preconditioner and scaling): assembles every
 * subdomain stiffness K^s = sum_e (Emin + rho_e^p (E0 - Emin)) K0 (Eq. 1), factorises
 * it, forms the explicit local dual operators F_s, the preconditioner blocks and the
 * coarse problem on the device.
 * rho: device [n_el] densities in [0, 1]. p >= 1, 0 < Emin < E0.
 * stream: a hipStream_t (NULL = the null stream); every later call on the context runs
 * on it. The context owns all of its device memory. */
feti_status feti_setup(const feti_mesh* mesh, const feti_partition* part, const feti_opts* opts,
                       const double* rho, double p, double E0, double Emin,
                       void* stream, feti_ctx** out);

/* Several independent designs in one context (their disjoint union as one decomposition):
 * every launch of setup and of the Krylov loop covers all designs at once, the FETI-DP coarse
 * matrix is block diagonal (one dense block per design) and the solve stops when every design
 * has reached tol in its own relative preconditioned residual. meshes/parts: host arrays of
 * n_designs entries (same dimension and Poisson ratio; FETI-DP only). rho, and the f, u,
 * dc_drho of later calls, concatenate the designs in order (offsets: feti_design_layout);
 * feti_compliance_and_grad writes one compliance per design (c: device [n_designs]).
 * S-FETI uses the union of the designs' direction groups (64 at most): each design searches
 * along its own groups, and since F couples no two designs the simultaneous directions of
 * different designs stay F-orthogonal. */
feti_status feti_setup_batched(int n_designs, const feti_mesh* meshes, const feti_partition* parts,
                               const feti_opts* opts, const double* rho, double p, double E0, double Emin,
                               void* stream, feti_ctx** out);

/* F*Lambda tile shapes. */
typedef struct {
    int max_red;              /* reduced-precision row blocks (of 16 rows) per tile, 1..32 */
    int max_d;                /* FP64 row blocks per tile, 1..16 */
    int xcd;                  /* 1: the tiles of one subdomain are placed on one XCD (shared L2) */
    int split_d;              /* FP64 row blocks per split-contraction tile (hybrid precision,
                                 subdomains that failed the round-off test), 1..4; 0 = no split
                                 contraction: plain FP64 tiles of up to max_d row blocks */
    double us;                /* in-solve F*Lambda kernel time with these shapes, microseconds */
    double us_default;        /* the same with the default shapes (32, 16, 1, 4) */
    int from_cache;           /* 1: read from the cache file, not timed */
    int fp64_first;           /* hybrid lists: 1 = the FP64 tiles of the subdomains that failed the
                                 round-off test lead the launch, 0 = they follow the reduced tiles */
} feti_tuning;

/* Autotuner of the F*Lambda tile shapes: times the context's in-solve F*Lambda (k = 64 columns,
 * the context's precision, hybrid lists included) over reps launches for every candidate in
 * max_red {32, 16} x max_d {16, 14, 12, 10, 8, 4} x xcd {1, 0} x split_d {4, 2} (hybrid lists:
 * split_d {4, 2, 1, 0} x fp64_first {0, 1}), keeps the fastest (a
 * change from the defaults must gain 2%) and applies it to every tile list of the context. cache_path (host string, optional): a JSON
 * file of earlier results keyed by (subdomains, n_b bucket of 32, precision, hybrid); a hit is
 * applied without timing, a miss is timed and written back. out: host, optional. Results of
 * F*Lambda do not depend on max_red, max_d, xcd or fp64_first (each row's contraction order is
 * fixed); split_d 0 against split_d > 0 changes the order of the FP64 rows of subdomains that failed
 * the round-off test (one sum against four partial sums), a difference at FP64 round-off. */
feti_status feti_autotune(feti_ctx* ctx, int reps, const char* cache_path, feti_tuning* out);

/* Applies the given F*Lambda tile shapes (as feti_autotune would after a search), for callers that
 * keep their own tuning. tune: host; its us, us_default and from_cache are not used. FETI_EINVAL
 * when a shape lies outside the ranges above. */
feti_status feti_set_tuning(feti_ctx* ctx, const feti_tuning* tune);

/* Ranges of design d (0 <= d < n_designs) in the concatenated arrays. */
feti_status feti_design_layout(feti_ctx* ctx, int d, feti_design* out);

/* Host out[n_designs]: each design's true relative residual sqrt(r_d^T M r_d) / eps0_d after the
 * last solve (r_d = the design's rows of d - F lambda, FP64). */
feti_status feti_design_residuals(feti_ctx* ctx, double* out, int cap);

/* New densities rho on the same mesh and partition (the SIMP law of Sec. 1, Eq. 1, re-evaluated
 * per element): repeats the setup of feti_setup from the assembly of every K^s (Sec. 2, Eq. 2-3)
 * through the factorisations, the local dual operators (Sec. 2.1 Eq. 7 / Sec. 2.2 Eq. 12), the
 * preconditioner blocks and scaling weights (Sec. 3.1, Eq. 13-15) and the coarse problem.
 * rho: device [n_el] in [0, 1]. Errors: FETI_EINVAL (null rho), FETI_ENOTSPD (a non-positive
 * pivot; the context must then be set up again before use). */
feti_status feti_update_rho(feti_ctx* ctx, const double* rho);

/* Solves K u = f (Eq. 2) by the configured FETI variant.
 * f: device [n_dof] global load (entries on clamped DOFs are ignored).
 * u: device [n_dof] output, the average of the subdomain copies.
 * lambda_init: device [n_lambda] warm start or NULL (FETI-DP: 0; TFETI: the
 * minimum-norm lambda with G lambda = e).
 * info: host, optional. Returns FETI_ENOCONV / FETI_EBREAKDOWN with u written. */
feti_status feti_solve(feti_ctx* ctx, const double* f, double* u, const double* lambda_init,
                       feti_info* info);

/* Compliance c = f^T u of the SIMP system (Sec. 1, Eq. 1-2: E_e = Emin + rho_e^p (E0 - Emin),
 * K(rho) u = f solved by the context's FETI variant, Sec. 2) and its gradient
 * dc/drho_e = -p rho_e^(p-1) (E0 - Emin) u_e^T K0 u_e (compliance is self-adjoint, so no second
 * solve), after feti_update_rho(rho) and feti_solve(f). Returns FETI_ENOCONV with c and dc
 * still written when the solve stopped at the iteration cap; callers that need a converged
 * gradient must check the status. A batched context writes one
 * compliance per design (c: device [n_designs]).
 * rho: device [n_el] or NULL (keep the current densities); f: device [n_dof] or NULL
 * (reuse the last load); c: device scalar; dc_drho: device [n_el]; u: device [n_dof] or NULL. */
feti_status feti_compliance_and_grad(feti_ctx* ctx, const double* rho, const double* f,
                                     double* c, double* dc_drho, double* u, feti_info* info);

/* The Lagrange multipliers lambda of the context's last solve (Sec. 2: the interface forces),
 * for a later warm start (feti_solve's lambda_init). lambda: device [n_lambda] output. FETI_EINVAL
 * before the first solve. */
feti_status feti_get_lambda(feti_ctx* ctx, double* lambda);

/* The local modes selected by opts.defl_modes at the last setup (deflation of local interface
 * modes; Sec. 6, item (ii)). mu: device [n_sub * defl_modes], eigenvalue i of subdomain s at
 * s * defl_modes + i in decreasing order, 0 past the modes selected for s; Y: device, optional,
 * [n_lambda x n_defl] row-major, the dual vectors y of the selected modes, subdomain by subdomain
 * (the vectors before F-orthonormalisation; the sign of each is arbitrary). FETI_EINVAL when the
 * context has no deflation. */
feti_status feti_get_deflation(feti_ctx* ctx, double* mu, double* Y);

/* One design update of the SIMP problem of Sec. 1 (minimum compliance c(rho) = f^T u under a bound
 * on the material volume, unit element volumes) by optimality criteria: with B_e(L) =
 * max(0, -dc_e) / L,
 *     rho_new_e = min(min(1, rho_e + move), max(max(rho_min, rho_e - move), rho_e B_e(L)^eta)),
 * and the multiplier L > 0 chosen so that sum_e rho_new_e = volfrac * n_el: the volume is
 * non-increasing in L, which is bracketed by 0 and max|dc| (doubled until the volume there is at
 * most the target) and bisected to a relative width of 1e-14 on per-workgroup partial volumes
 * summed on the host in a fixed order. rho, dc: device [n_el] (dc from feti_compliance_and_grad);
 * rho_new: device [n_el] output (may alias neither input); lagrange: host, optional, receives L.
 * Single-design contexts; needs 0 <= rho_min < volfrac <= 1, move > 0, eta > 0 (FETI_EINVAL
 * otherwise). Synchronises the context's stream once per bisection step. */
feti_status feti_oc_update(feti_ctx* ctx, const double* rho, const double* dc, double volfrac, double move,
                           double eta, double rho_min, double* rho_new, double* lagrange);

feti_status feti_destroy(feti_ctx* ctx);

const char* feti_last_error(void);

/* ---- entry points of single steps of the Krylov loop (kernel-level access) ---- */

feti_status feti_get_sizes(feti_ctx* ctx, feti_sizes* out);

/* Q = F Lambda for a block of k directions (Sec. 2.1 Eq. 7: F = B K^+ B^T; Sec. 2.2 Eq. 12
 * with u_c condensed: F_rr + F_rc Kbar_cc^{-1} F_rc^T). Lambda, Q: device [n_lambda x k]
 * row-major FP64; precision selects the arithmetic of the local products
 * (FP64, FP32 or BF16 split into hi + lo with three products). For FETI-DP with the
 * context's own reduced precision, subdomains whose F_s failed the setup's round-off test
 * (Cholesky pivots of F_s and of its rounding differing by more than 2 percent) run in FP64;
 * or-ing FETI_PURE forces every subdomain to the reduced precision. 1 <= k <= 64. */
feti_status feti_apply_F(feti_ctx* ctx, int k, int precision, const double* Lambda, double* Q);

/* The product of feti_apply_F (same arguments, same kernels, bit-identical Q) for callers that
 * cannot allocate device memory or wait on the device: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc. It calls no allocation routine and does not
 * synchronise or time: the work is only enqueued on the context's stream. Its work buffers (the
 * local products, the corner rows and the coarse vectors: 8 * k * (sum n_b + sum n_c + 2 n_cg)
 * bytes, each part rounded up to 256) live in a fixed 16 MiB device array that every GPU holds
 * once for the life of the process; a larger request returns FETI_EINVAL and enqueues nothing.
 * All calls on one GPU share that array, so calls that overlap in time on one GPU (other
 * streams, other contexts, other host threads) race; serialise them. */
feti_status feti_apply_F_noalloc(feti_ctx* ctx, int k, int precision, const double* Lambda, double* Q);

/* Z = [.., B~^s S~^s B~^sT r, ..] (Sec. 3.1 Eq. 13, Algorithm 1): r device [n_lambda];
 * Z device [n_lambda x n_groups] (one_column = 0) or [n_lambda] summed (one_column = 1).
 * one_column or-ed with FETI_PRECOND_FP32: S~^s from its FP32 copy (a context set up with
 * precond_fp32 = 1; FETI_EINVAL otherwise), FP64 products and sums. */
feti_status feti_apply_precond(feti_ctx* ctx, const double* r, double* Z, int one_column);

/* Y <- P Y with P = I - G^T (G G^T)^{-1} G (TFETI, Sec. 3.3); identity for FETI-DP.
 * Y device [n_lambda x k], in place. */
feti_status feti_project(feti_ctx* ctx, int k, double* Y);

/* d (right-hand side of the lambda system) and lambda_0 for load f:
 * TFETI d = B K^+ f (c = 0), lambda_0 = G^T (G G^T)^{-1} e; FETI-DP d = d_r - F_rc
 * Kbar_cc^{-1} fbar_c, lambda_0 = 0. f device [n_dof]; d, lambda0 device [n_lambda]. */
feti_status feti_rhs(feti_ctx* ctx, const double* f, double* d, double* lambda0);

/* Copies one local matrix of subdomain s to host memory (for checking against the
 * oracle). what: 0 = F_s [n_b x n_b]; 1 = S~^s preconditioner block [n_b x n_b];
 * 2 = F_rc^s [n_b x n_c]; 3 = Kbar_cc^s [n_c x n_c]; 4 = scaling weight of every lambda row on
 * each side [n_lambda x 2] (s ignored); 5 = the assembled Kbar_cc of design s [n_cg x n_cg of that
 * design] (s = 0 for a single design: the whole coarse matrix);
 * 6 = diagonal of K^s [n_loc]. out: host, capacity cap doubles; rows/cols: host, receive the shape. */
feti_status feti_get_local(feti_ctx* ctx, int s, int what, double* out, long long cap,
                           int* rows, int* cols);

/* Milliseconds of the last call's device work, measured with HIP events on the context's
 * stream: what 0 = last feti_apply_F (the local product kernel only), 1 = last feti_apply_F
 * total, 2 = last feti_setup / feti_update_rho, 3 = last feti_solve. */
feti_status feti_last_timing(feti_ctx* ctx, int what, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* FETI_H */
