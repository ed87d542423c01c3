"""Deflation of local interface modes on the HIP path (the further-work item (ii) of Sec. 6, read as
in oracle/deflation.py: the largest eigenpairs of every subdomain's local preconditioned operator,
taken up to a 5% spectral gap, removed from the iteration), against the oracle:

* the local eigenvalues selected per subdomain (count and values) and the dual vectors they give
  (the span of each subdomain's columns: eigenvectors are unique only up to sign);
* deflated FETI-DP with PCG, full orthogonalisation and S-FETI on the layered grid (Sec. 4.1): u
  against the global direct solution, the iteration count at 1e-6 against the oracle's deflated
  run (within 2), and below the plain run's (PCG and FO at most half);
* a Beta-distributed design (the workload family of the benchmark) with FP32 F*Lambda;
* the option's limits (Total FETI, recycling) are refused."""
import numpy as np
import pytest

import workloads
from oracle import deflation, fem, feti as ofeti, krylov

torch = pytest.importorskip("torch")
feti = pytest.importorskip("paper_2111_11728_amd.feti")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
M_MODES = 8


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _ctx(prob, **kw):
    return feti.Context(feti.Spec(prob, method="fetidp", scaling="k", precond="dirichlet", **kw), _t(prob.rho))


@pytest.fixture(scope="module")
def layered():
    prob = workloads.layered_grid()
    op = ofeti.FETIDP(prob, "dirichlet", "k")
    Y, mus = deflation.deflation_space(op, M_MODES)
    return prob, op, Y, mus


def test_local_modes_against_oracle(layered):
    prob, op, Y_ref, mus = layered
    print("case deflation modes layered_grid", flush=True)
    ctx = _ctx(prob, krylov="sfeti", defl_modes=M_MODES)
    sz = ctx.sizes
    ns = sz["n_sub"]
    mu = torch.zeros(ns * M_MODES, dtype=torch.float64, device=DEV)
    Y = torch.zeros(op.n_lambda, max(1, sz["n_defl"]), dtype=torch.float64, device=DEV)
    ctx.feti_get_deflation(mu, Y)
    ctx.close()
    mu = mu.cpu().numpy().reshape(ns, M_MODES)
    Y = Y.cpu().numpy()[:, :sz["n_defl"]]
    assert sz["n_defl"] == Y_ref.shape[1] == sum(len(m) for m in mus)
    c0 = 0
    for s in range(ns):
        k = len(mus[s])
        print(f"  subdomain {s}: {k} modes, oracle mu {np.array2string(mus[s], precision=4)}", flush=True)
        assert np.count_nonzero(mu[s]) == k
        assert np.allclose(mu[s, :k], mus[s], rtol=1e-8, atol=0.0)
        A, B = Y[:, c0:c0 + k], Y_ref[:, c0:c0 + k]
        # each oracle vector lies in the span of the GPU's (and the dimensions agree)
        q, _ = np.linalg.qr(A)
        res = np.linalg.norm(B - q @ (q.T @ B), axis=0) / np.linalg.norm(B, axis=0)
        assert res.max() <= 1e-6, (s, res)
        c0 += k
    assert sz["n_defl_kept"] == sz["n_defl"]


@pytest.mark.parametrize("kind", ["pcg", "fo", "sfeti"])
def test_deflated_solve_against_oracle(layered, kind):
    prob, op, Y_ref, _ = layered
    print(f"case deflated solve layered_grid {kind}", flush=True)
    ref = krylov.solve(op, kind, tol=1e-6, Y=Y_ref)
    plain = krylov.solve(op, kind, tol=1e-6)
    f = _t(prob.load())
    u_star = fem.solve_problem(prob)
    its = {}
    for tol in (1e-6, 1e-10):
        ctx = _ctx(prob, krylov=kind, tol=tol, defl_modes=M_MODES)
        u = torch.zeros(prob.n_dof, dtype=torch.float64, device=DEV)
        info = ctx.feti_solve(f, u)
        ctx.close()
        its[tol] = info["iters"]
        err = np.linalg.norm(u.cpu().numpy() - u_star) / np.linalg.norm(u_star)
        print(f"  tol {tol:.0e}: {info['iters']} iterations (oracle {ref.iters} deflated, {plain.iters} plain), "
              f"u error {err:.1e}", flush=True)
        if tol == 1e-10:
            assert err <= 1e-8
    assert abs(its[1e-6] - ref.iters) <= 2
    # the oracle, deflated against plain: PCG 19 / 88, FO 18 / 61, S-FETI 11 / 16
    assert its[1e-6] <= (plain.iters // 2 if kind != "sfeti" else plain.iters - 3)


def test_beta_design_mixed_precision():
    prob = workloads.beta_2d(0, nsub=(4, 4), m=16)
    print("case deflation beta 4x4 of 16 fp32", flush=True)
    op = ofeti.FETIDP(prob, "dirichlet", "k")
    Y_ref, _ = deflation.deflation_space(op, 4)
    ref = krylov.solve(op, "sfeti", tol=1e-8, Y=Y_ref)
    f = _t(prob.load())
    u_star = fem.solve_problem(prob)
    ctx = _ctx(prob, krylov="sfeti", tol=1e-8, precision="fp32", defl_modes=4)
    u = torch.zeros(prob.n_dof, dtype=torch.float64, device=DEV)
    info = ctx.feti_solve(f, u)
    n_defl = ctx.sizes["n_defl"]
    ctx.close()
    err = np.linalg.norm(u.cpu().numpy() - u_star) / np.linalg.norm(u_star)
    print(f"  {n_defl} modes (oracle {Y_ref.shape[1]}), {info['iters']} iterations (oracle {ref.iters}), "
          f"u error {err:.1e}", flush=True)
    assert n_defl == Y_ref.shape[1]
    assert err <= 1e-6
    assert abs(info["iters"] - ref.iters) <= 2


def test_refused_combinations():
    prob = workloads.cantilever_tfeti(0)
    with pytest.raises(feti.FetiError):
        feti.Context(feti.Spec(prob, method="tfeti", krylov="sfeti", defl_modes=4), _t(prob.rho))
    with pytest.raises(feti.FetiError):
        feti.Context(feti.Spec(prob, method="fetidp", krylov="sfeti", defl_modes=4, recycle=1), _t(prob.rho))
    with pytest.raises(feti.FetiError):
        feti.Context(feti.Spec(prob, method="fetidp", krylov="sfeti", defl_modes=9), _t(prob.rho))
