"""Pins of the oracle's finite-element layer against hand-derived closed forms,
invariants and finite differences (no GPU)."""
import numpy as np
import pytest

import workloads
from oracle import fem

NU = 0.3


def test_q4_entries_closed_form():
    # unit square, E = 1, plane stress; corners (0,0),(1,0),(0,1),(1,1), DOFs (u, v)
    K = fem.element_stiffness(2, NU)
    c = 1.0 / (1.0 - NU ** 2)
    assert K[0, 0] == pytest.approx(c * (3 - NU) / 6, rel=1e-14)          # u1,u1
    assert K[0, 0] == pytest.approx(0.4945054945054945, rel=1e-12)
    assert K[0, 1] == pytest.approx(1.0 / (8 * (1 - NU)), rel=1e-14)      # u1,v1
    assert K[0, 2] == pytest.approx(-c * (3 + NU) / 12, rel=1e-14)        # u1,u2
    assert K[0, 6] == pytest.approx(-c * (3 - NU) / 12, rel=1e-14)        # u1,u4 (opposite corner)
    assert K[0, 3] == pytest.approx(c * (3 * NU - 1) / 8, rel=1e-14)      # u1,v2


def test_hex8_entries_closed_form():
    K = fem.element_stiffness(3, NU)
    lam = NU / ((1 + NU) * (1 - 2 * NU))
    mu = 1 / (2 * (1 + NU))
    D11 = lam + 2 * mu
    assert K[0, 0] == pytest.approx((D11 + 2 * mu) / 9, rel=1e-14)
    assert K[0, 0] == pytest.approx(0.23504273504273504, rel=1e-12)
    assert K[0, 1] == pytest.approx((lam + mu) / 12, rel=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_symmetric_with_rigid_null_space(dim):
    K = fem.element_stiffness(dim, NU)
    assert np.allclose(K, K.T, atol=1e-15)
    ev = np.linalg.eigvalsh(K)
    n_rbm = 3 if dim == 2 else 6
    assert np.all(np.abs(ev[:n_rbm]) < 1e-12)
    assert ev[n_rbm] > 1e-3
    # translations give zero forces
    for a in range(dim):
        t = np.zeros(K.shape[0])
        t[a::dim] = 1.0
        assert np.abs(K @ t).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_element_patch_energy(dim):
    """Linear displacement u = A x gives energy u^T K u = eps^T D eps on a unit element."""
    rng = np.random.default_rng(1)
    A = rng.standard_normal((dim, dim))
    K = fem.element_stiffness(dim, NU)
    corners = np.array(fem.corner_offsets(dim), dtype=float)
    u = (corners @ A.T).ravel()
    S = 0.5 * (A + A.T)
    if dim == 2:
        eps = np.array([S[0, 0], S[1, 1], 2 * S[0, 1]])
    else:
        eps = np.array([S[0, 0], S[1, 1], S[2, 2], 2 * S[1, 2], 2 * S[0, 2], 2 * S[0, 1]])
    D = fem.material_matrix(dim, NU)
    assert u @ K @ u == pytest.approx(eps @ D @ eps, rel=1e-12)


def test_global_patch_and_assembly():
    """A linear field on a heterogeneous-free mesh leaves zero force at interior nodes;
    every element contributes its own block (two-element hand check)."""
    nel = (5, 4)
    K = fem.assemble_global(nel, NU, np.ones(20)).toarray()
    nn = (6, 5)
    X, Y = np.meshgrid(np.arange(nn[0]), np.arange(nn[1]))
    u = np.zeros(2 * 30)
    u[0::2] = (0.3 * X + 0.1 * Y).ravel()
    u[1::2] = (-0.2 * X + 0.5 * Y).ravel()
    fint = K @ u
    interior = [(ix + nn[0] * iy) for iy in range(1, nn[1] - 1) for ix in range(1, nn[0] - 1)]
    for nd in interior:
        assert abs(fint[2 * nd]) < 1e-12 and abs(fint[2 * nd + 1]) < 1e-12
    K2 = fem.assemble_global((2, 1), NU, np.array([1.0, 2.0])).toarray()
    Ke = fem.element_stiffness(2, NU)
    ref = np.zeros((12, 12))
    for e, (E, nodes) in enumerate([(1.0, [0, 1, 3, 4]), (2.0, [1, 2, 4, 5])]):
        d = np.array([[2 * n, 2 * n + 1] for n in nodes]).ravel()
        ref[np.ix_(d, d)] += E * Ke
    assert np.allclose(K2, ref, atol=1e-15)


def test_simp_law():
    E = fem.simp_modulus(np.array([0.0, 0.5, 1.0]), 3.0, 1.0, 1e-6)
    assert E[0] == 1e-6 and E[2] == 1.0
    assert E[1] == pytest.approx(1e-6 + 0.125 * (1 - 1e-6))


def test_compliance_identities_and_fd_gradient():
    prob = workloads.cantilever_tfeti(3, nsub=(2, 1), m=4)
    u = fem.solve_problem(prob)
    f = prob.load()
    E = fem.simp_modulus(prob.rho, prob.p, prob.E0, prob.Emin)
    K = fem.assemble_global(prob.nel, prob.nu, E)
    c = fem.compliance(f, u)
    assert c == pytest.approx(u @ (K @ u), rel=1e-12)
    g = fem.compliance_gradient(prob, u)
    Kmin = fem.assemble_global(prob.nel, prob.nu, np.full(prob.n_el, prob.Emin))
    assert np.dot(prob.rho, g) == pytest.approx(-prob.p * (c - u @ (Kmin @ u)), rel=1e-10)
    h = 1e-4
    for e in [0, 5, 17, 30]:
        rp = prob.rho.copy(); rp[e] += h
        rm = prob.rho.copy(); rm[e] -= h
        cp = fem.compliance(f, fem.solve_problem(workloads.Problem(2, prob.nel, prob.cuts, rp)))
        cm = fem.compliance(f, fem.solve_problem(workloads.Problem(2, prob.nel, prob.cuts, rm)))
        assert (cp - cm) / (2 * h) == pytest.approx(g[e], rel=1e-5, abs=1e-6 * abs(g).max())


def test_load_and_clamp_conventions():
    f = workloads.point_load(2, (32, 16))
    node = 32 + 33 * 8
    assert f[2 * node + 1] == -1.0 and np.count_nonzero(f) == 1
    fx = workloads.clamped_dofs(2, (32, 16))
    assert fx.size == 2 * 17 and set(fx[0::2] // 2) == {33 * j for j in range(17)}
    f3 = workloads.point_load(3, (4, 4, 4))
    node3 = 4 + 5 * 2 + 25 * 2
    assert f3[3 * node3 + 1] == -1.0
