"""Pins of the oracle's decomposition layer: interface sizes by hand counting,
continuity of the direct solution, admissible scaling (Sec. 3.1, Eq. 14) and the
k-scaling / multiplicity equivalence for homogeneous material (no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from oracle import fem, feti, topology


def count_2d(Sx, Sy, m):
    """Hand count for a uniform 2D grid of Sx x Sy subdomains of m x m elements with
    the x = 0 edge clamped: TFETI rows, FETI-DP rows and corner DOFs."""
    ny = Sy * m
    # TFETI: clamped copies (left edge nodes, shared ones counted per subdomain) x 2 DOFs
    dirichlet = 2 * ((ny + 1) + (Sy - 1))
    cross = (Sx - 1) * (Sy - 1)                    # interior cross-points, m = 4 -> 6 pairs
    vert_nodes = (Sx - 1) * (ny + 1)               # nodes on vertical interfaces
    hor_nodes = (Sy - 1) * (Sx * m)                # nodes on horizontal interfaces, x > 0
    pair2 = vert_nodes + hor_nodes - 2 * cross     # every cross-point sits on both families
    tfeti = dirichlet + 2 * (pair2 + 6 * cross)
    # FETI-DP: corners = subdomain vertices shared by >= 2 subdomains, not on x = 0
    corners = (Sx) * (Sy + 1) - 2                  # columns x = 1..Sx of vertex grid, minus the two outer right corners
    dual_vert = (Sx - 1) * (ny + 1 - (Sy + 1))     # vertical interface nodes minus vertices
    dual_hor = (Sy - 1) * (Sx * m + 1 - 1 - Sx)    # horizontal: minus clamped x=0 and Sx vertices
    return tfeti, 2 * (dual_vert + dual_hor), 2 * corners


@pytest.mark.parametrize("Sx,Sy,m", [(4, 2, 8), (8, 4, 32), (3, 3, 4), (2, 1, 3)])
def test_interface_sizes(Sx, Sy, m):
    prob = workloads.cantilever_tfeti(0, nsub=(Sx, Sy), m=m)
    dec = topology.decompose(prob)
    cons = topology.tfeti_constraints(dec)
    split, dp = topology.fetidp_split(dec)
    n_t, n_dp, n_cg = count_2d(Sx, Sy, m)
    assert cons.n_rows == n_t
    assert dp.n_rows == n_dp
    assert split.corner_dofs.size == n_cg


def test_survey_size_table_c1():
    prob = workloads.cantilever_tfeti(0)
    dec = topology.decompose(prob)
    cons = topology.tfeti_constraints(dec)
    assert cons.n_rows == 226
    assert sum(b.size ** 2 for b in cons.bset) == 17312
    split, dp = topology.fetidp_split(dec)
    nb = [b.size for b in dp.bset]
    assert (dp.n_rows, split.corner_dofs.size, max(nb), min(nb), sum(x * x for x in nb)) == (140, 20, 42, 28, 10192)


def test_3d_counts_small():
    """2x2x2 subdomains of 2^3 elements, x = 0 face clamped: FETI-DP rows counted by hand.
    Dual nodes: face nodes (m = 2) and edge nodes (m = 4, 6 pairs)."""
    prob = workloads.modular_3d(0, nsub=(2, 2, 2), m=2)
    dec = topology.decompose(prob)
    split, dp = topology.fetidp_split(dec)
    # grid of nodes 5^3; interface planes x=2, y=2, z=2; vertices at coordinates in {0,2,4}
    n_dual_rows = 0
    for ix in range(5):
        for iy in range(5):
            for iz in range(5):
                on = [c == 2 for c in (ix, iy, iz)]
                m = 2 ** sum(on)
                if m < 2 or ix == 0:
                    continue
                vertex = all(c in (0, 2, 4) for c in (ix, iy, iz))
                if vertex:
                    continue
                n_dual_rows += 3 * m * (m - 1) // 2
    assert dp.n_rows == n_dual_rows
    n_corner_nodes = sum(1 for ix in (2, 4) for iy in (0, 2, 4) for iz in (0, 2, 4)
                         if 2 ** sum(c == 2 for c in (ix, iy, iz)) >= 2)
    assert split.corner_dofs.size == 3 * n_corner_nodes


def _torn(dec, u):
    return [u[sd.dofs] for sd in dec.subs]


def test_direct_solution_satisfies_constraints():
    """B u = 0 (TFETI: continuity and clamps, Eq. 4) and B_r u_r = 0 (Eq. 10) for the
    subdomain restrictions of the global direct solution."""
    prob = workloads.cantilever_tfeti(2, nsub=(3, 3), m=4)
    u = fem.solve_problem(prob)
    dec = topology.decompose(prob)
    cons = topology.tfeti_constraints(dec)
    us = _torn(dec, u)
    assert np.abs(sum(cons.B[s] @ us[s] for s in range(9))).max() < 1e-14
    split, dp = topology.fetidp_split(dec)
    assert np.abs(sum(dp.B[s] @ us[s][split.r[s]] for s in range(9))).max() < 1e-14
    # a perturbed copy is caught
    us[4] = us[4] + 1e-3
    assert np.abs(sum(cons.B[s] @ us[s] for s in range(9))).max() > 1e-4


@pytest.mark.parametrize("method", ["tfeti", "fetidp"])
@pytest.mark.parametrize("kind", ["mult", "k"])
def test_admissible_scaling(method, kind):
    """sum_s B^s B~^sT B^j = B^j for every j (Sec. 3.1, Eq. 14), redundant cross-points included."""
    prob = workloads.cantilever_tfeti(5, nsub=(3, 3), m=3)
    op = feti.TFETI(prob, "lumped", kind) if method == "tfeti" else feti.FETIDP(prob, "lumped", kind)
    B = op.cons.B
    W = [sp.diags(w) for w in op.w]
    M = sum(B[s] @ (W[s] @ B[s]).T for s in range(len(B)))
    for j in range(len(B)):
        assert abs(M @ B[j] - B[j]).max() < 1e-13


def test_kscaling_is_multiplicity_for_homogeneous():
    prob = workloads.cantilever_tfeti(0, nsub=(3, 3), m=3)
    prob.rho[:] = 1.0
    a = feti.TFETI(prob, "lumped", "k")
    b = feti.TFETI(prob, "lumped", "mult")
    for wa, wb in zip(a.w, b.w):
        assert np.allclose(wa, wb, atol=1e-14)


def test_rigid_body_modes_span_kernel():
    prob = workloads.cantilever_tfeti(0, nsub=(2, 2), m=3)
    op = feti.TFETI(prob)
    for Ks, R in zip(op.K, op.R):
        assert np.abs(Ks @ R).max() < 1e-12
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-13)
        ev = np.linalg.eigvalsh(Ks.toarray())
        assert ev[2] < 1e-12 * ev[-1] and ev[3] > 1e-10 * ev[-1]


def test_group_assignment():
    g = workloads.group_of_subdomains((16, 16), (2, 2))
    assert g.max() == 63 and np.bincount(g).min() == 4
    assert g[0] == g[1] == g[16] == g[17] == 0 and g[2] == 1 and g[32] == 8
    g32 = workloads.group_of_subdomains((16, 16), (4, 2))
    assert g32.max() == 31 and g32[3] == 0 and g32[4] == 1 and g32[16] == 0 and g32[32] == 4
