"""Pins of the oracle's deflation of local interface modes (the further-work item (ii) of Sec. 6,
read as in oracle/deflation.py), no GPU:

* the local eigenvalues mu against the nonzero eigenvalues of the dense local product P_s F_s
  (a general eigensolver on the product, not the symmetric reduction the oracle takes), and the
  dual vectors y as its eigenvectors;
* deflated S-FETI, fully orthogonalised PCG and PCG reach the global direct solution (FETI-DP
  and TFETI);
* a deflation space spanning the whole dual space solves the problem before the first iteration;
* after the start correction the residual is orthogonal to the deflation space;
* the selection takes a cluster of equal eigenvalues whole or not at all;
* on the layered grid the orthogonalised PCG needs far fewer iterations with the 8 largest local
  modes of every subdomain deflated (measured here: FETI-DP 61 -> 18)."""
import numpy as np
import pytest

import workloads
from oracle import deflation, fem, feti, krylov


def _op(prob, method, precond="dirichlet"):
    return feti.FETIDP(prob, precond, "k") if method == "fetidp" else feti.TFETI(prob, precond, "k")


@pytest.mark.parametrize("method", ["fetidp", "tfeti"])
def test_local_modes_are_eigenpairs_of_the_local_preconditioned_operator(method):
    prob = workloads.inclusion_grid(nsub=(3, 2), m=6)
    op = _op(prob, method)
    for s in range(len(op.dec.subs)):
        mu, _, Y = deflation.local_modes(op, s, 5, gap=0.0)
        Bb = op.cons.Bb[s]
        rows = np.unique(Bb.nonzero()[0])
        Bs = Bb[rows].toarray()
        w = op.w[s][rows]
        P = (w[:, None] * Bs) @ np.asarray(op.S[s]) @ (Bs.T * w[None, :])
        F = Bs @ op.F_local[s] @ Bs.T
        ev = np.linalg.eigvals(P @ F)
        ev = np.sort(ev.real[np.abs(ev.real) > 1e-9 * np.abs(ev).max()])[::-1]
        assert np.allclose(mu, ev[:mu.size], rtol=1e-9, atol=0.0), (s, mu, ev[:mu.size])
        for i in range(mu.size):
            y = Y[rows, i]
            assert np.linalg.norm(P @ (F @ y) - mu[i] * y) <= 1e-9 * mu[i] * np.linalg.norm(y)
        assert np.all(Y[np.setdiff1d(np.arange(op.n_lambda), rows)] == 0.0)


@pytest.mark.parametrize("method,kind", [("fetidp", "sfeti"), ("fetidp", "fo"), ("fetidp", "pcg"), ("tfeti", "sfeti"),
                                         ("tfeti", "fo"), ("tfeti", "pcg")])
def test_deflated_solve_reaches_the_direct_solution(method, kind):
    prob = workloads.cantilever_tfeti(1, nsub=(3, 2), m=6)
    op = _op(prob, method)
    Y, _ = deflation.deflation_space(op, 3)
    res = krylov.solve(op, kind, tol=1e-12, Y=Y)
    assert res.converged
    u, _ = op.recover(res.lam)
    u_star = fem.solve_problem(prob)
    assert np.linalg.norm(u - u_star) <= 1e-8 * np.linalg.norm(u_star)


def test_selection_takes_clusters_whole():
    mu = np.array([5.0, 4.0, 3.0, 3.0, 3.0, 1.0])
    assert deflation.select_count(mu, 3) == 2          # the cluster at 3 would be cut
    assert deflation.select_count(mu, 5) == 5
    assert deflation.select_count(mu, 8) == 6          # past the spectrum mu_{k+1} = 0
    assert deflation.select_count(mu, 8, tau=3.5) == 2
    assert deflation.select_count(np.full(4, 2.0), 2) == 0


def test_full_space_deflation_solves_before_iterating():
    prob = workloads.cantilever_tfeti(2, nsub=(2, 2), m=4)
    op = _op(prob, "fetidp")
    Y = np.eye(op.n_lambda)
    res = krylov.solve(op, "sfeti", tol=1e-10, Y=Y)
    assert res.converged and res.iters == 0
    u, _ = op.recover(res.lam)
    u_star = fem.solve_problem(prob)
    assert np.linalg.norm(u - u_star) <= 1e-9 * np.linalg.norm(u_star)


@pytest.mark.parametrize("method", ["fetidp", "tfeti"])
def test_residual_orthogonal_to_the_deflation_space(method):
    prob = workloads.inclusion_grid(nsub=(3, 3), m=6)
    op = _op(prob, method)
    Y, _ = deflation.deflation_space(op, 4, gap=0.0)   # the selection is not what is tested here
    r0 = op.project((op.d - op.apply_F(op.lambda0()[:, None])[:, 0])[:, None])[:, 0]
    Wd, Qd, lt, r = krylov.deflate(op, Y, r0.copy())
    W = np.hstack(Wd)
    # F-orthonormal basis
    assert np.allclose(W.T @ np.hstack(Qd), np.eye(W.shape[1]), atol=1e-9)
    # the correction is consistent: r = P (d - F (lam0 + lt))
    r_chk = op.project((op.d - op.apply_F((op.lambda0() + lt)[:, None])[:, 0])[:, None])[:, 0]
    assert np.linalg.norm(r - r_chk) <= 1e-10 * np.linalg.norm(r0)
    # Galerkin condition on the span of P Y
    PY = op.project(Y)
    assert np.abs(PY.T @ r).max() <= 1e-9 * np.abs(PY).max() * np.linalg.norm(r0)


@pytest.mark.parametrize("kind", ["fo", "pcg"])
def test_fewer_iterations_on_the_layered_grid(kind):
    prob = workloads.layered_grid()
    op = _op(prob, "fetidp")
    plain = krylov.solve(op, kind, tol=1e-6)
    Y, mus = deflation.deflation_space(op, 8)
    defl = krylov.solve(op, kind, tol=1e-6, Y=Y)
    assert plain.converged and defl.converged
    assert defl.iters <= plain.iters // 2, (plain.iters, defl.iters)
