// Integer topology of a FETI decomposition on a structured grid (host only).
//
// Builds, once per (mesh, partition, method), everything that does not depend on the
// densities: the class of every subdomain-local DOF (interior i, interface b touched by
// the constraint rows, FETI-DP corner c, clamped x), the Lagrange-multiplier rows of
// TFETI (Sec. 2.1, Eq. 4: pairwise gluing plus one Dirichlet row per subdomain copy of a
// clamped DOF) or of FETI-DP (Sec. 2.2, Eq. 10: pairwise gluing of the non-corner DOFs),
// the corner numbering of the primal vector u_c (Eq. 9), the gather lists used by
// B^T Lambda, and the half-bandwidth of every interior block K_ii.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "classes.hpp"
#include "feti.h"

namespace feti {

struct Plan {
    int dim = 2, dpn = 2, method = FETI_DP;
    int nel[3] = {1, 1, 1}, nsub[3] = {1, 1, 1};
    int n_sub = 0, n_el = 0, n_nodes = 0, n_dof = 0;
    double nu = 0.3;
    std::vector<int> cuts[3];
    // per axis and global node coordinate: first subdomain index along the axis that
    // contains the coordinate, and how many (1 or 2)
    std::vector<int> ax_first[3], ax_cnt[3];

    // ---- per subdomain ----
    std::vector<int> lo, nn;              // [3*n_sub] first element / local nodes per axis
    std::vector<int> n_loc, n_i, n_b, n_c, band, grp;
    std::vector<int64_t> off_loc, off_i, off_b, off_c;  // prefix sums, size n_sub+1
    int n_groups = 0;
    int group[3] = {1, 1, 1};

    // ---- per local DOF, concatenated over subdomains (size off_loc[n_sub]) ----
    std::vector<int8_t> lcls;             // CLS_*
    std::vector<int> lidx;                // index inside its class list
    std::vector<int> lglob;               // global DOF
    std::vector<int8_t> lown;             // 1 if this subdomain is the lowest one holding the DOF

    // class lists (local DOF numbers), concatenated
    std::vector<int> i_loc, b_loc, c_loc;
    std::vector<int> c_glob;              // per corner DOF of a subdomain: global corner index

    // ---- lambda rows ----
    int n_lambda = 0;
    std::vector<int> row_s, row_j;        // [2*n_lambda]: subdomain and b-index per side (-1: no side)
    std::vector<int8_t> row_sg;           // [2*n_lambda] sign per side
    std::vector<int> row_sh;              // [n_lambda] shared-DOF id (-1 for Dirichlet rows)
    std::vector<int> sh_ptr, sh_s, sh_l;  // shared DOF -> members (subdomain, local DOF)
    // gather lists: b DOF (global b index off_b[s]+j) -> rows touching it, with sign
    std::vector<int> bg_ptr, bg_row;
    std::vector<int8_t> bg_sg;

    // ---- corners (FETI-DP) ----
    int n_cg = 0;
    std::vector<int> corner_dofs;         // global DOF of each corner index
    std::vector<int> cc_ptr, cc_s, cc_j;  // corner index -> (subdomain, c-index) members

    // ---- TFETI ----
    int n_rbm = 0, n_alpha = 0;

    int64_t sum_nb2() const;
    int64_t sum_nb_nc() const;
};

// Returns "" on success or an error message.
std::string build_plan(const feti_mesh* mesh, const feti_partition* part, const feti_opts* opts,
                       Plan& P);

// Adaptive choice of further FETI-DP primal nodes from the densities (2D; 3D: none): along every
// edge shared by two subdomains (end vertices excluded), runs of nodes whose stiffness (sum of the
// moduli Emin + rho^p (E0 - Emin) of their elements) is at least theta times the edge's largest;
// the cap runs of largest total stiffness give their middle nodes. out: sorted global nodes.
std::string adaptive_primal(const feti_mesh* mesh, const feti_partition* part, const double* rho, double p,
                            double E0, double Emin, double theta, int cap, std::vector<int>& out);

// One design inside a plan that holds several independent designs (their disjoint union):
// the ranges of its subdomains, elements, nodes, DOFs, lambda rows, corners and S-FETI
// direction groups in the union's numbering, and its own structured grid.
struct DesignMeta {
    int sub0 = 0, n_sub = 0;
    int64_t el0 = 0, n_el = 0, node0 = 0, n_nodes = 0, dof0 = 0, n_dof = 0;
    int lam0 = 0, n_lambda = 0, cg0 = 0, n_cg = 0, grp0 = 0, n_groups = 0;
    int n_rows = 0;   // lambda rows reserved for the design (n_lambda, padded when segmented)
    int nel[3] = {1, 1, 1}, nsub[3] = {1, 1, 1};
    std::vector<int> ax_first[3], ax_cnt[3];
};

// The union of nd designs (same dimension, method and options) as one decomposition: the
// per-design plans concatenated with offsets. The union's nel/nsub/ax_* are those of design 0
// when nd == 1 and unused otherwise (per-design data is in D).
// segmented: every design keeps its own direction groups (numbered from 0; the union's n_groups
// is their maximum) and its lambda rows are padded with empty rows (no side) to a multiple of 256.
std::string build_plan_batched(int nd, const feti_mesh* meshes, const feti_partition* parts, const feti_opts* opts,
                               Plan& U, std::vector<DesignMeta>& D, bool segmented = false);

}  // namespace feti
