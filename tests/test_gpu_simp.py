"""The SIMP design update and the warm-started design loop on the HIP path (the application of
Sec. 1: minimum compliance under a volume bound, Eq. 1-2), against the oracle:

* feti_oc_update (optimality criteria) against oracle.simp.oc_update on the same seeded
  densities and sensitivities: the multiplier of the volume bound and every updated density;
* a short design loop (compliance and gradient, update with a move limit of 0.02, next design) with
  warm-started multipliers
  (opts.warm_start): every design's u against the global direct solution of that design, the
  compliance against the oracle's, and the warm-started solves needing fewer iterations than cold
  ones, for FETI-DP and Total FETI (whose warm start must be made feasible for G lambda = e)."""
import numpy as np
import pytest

import workloads
from oracle import fem, simp

torch = pytest.importorskip("torch")
feti = pytest.importorskip("paper_2111_11728_amd.feti")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("n_case", [0, 1])
def test_oc_update_against_oracle(n_case):
    prob = [workloads.cantilever_tfeti(4), workloads.modular_2d(2, nsub=(4, 4), m=16)][n_case]
    rng = np.random.default_rng(40 + n_case)
    rho = np.clip(prob.rho, 0.0, 1.0)
    dc = -rng.gamma(0.5, 2.0, prob.n_el) * np.maximum(rho, 1e-3) ** 2
    print(f"case oc update {prob.name}", flush=True)
    ctx = feti.Context(feti.Spec(prob, method="fetidp"), _t(rho))
    out = torch.zeros(prob.n_el, dtype=torch.float64, device=DEV)
    L = ctx.feti_oc_update(_t(rho), _t(dc), out, 0.45, move=0.2, eta=0.5, rho_min=1e-3)
    ctx.close()
    ref, L_ref = simp.oc_update(rho, dc, 0.45, move=0.2, eta=0.5, rho_min=1e-3)
    new = out.cpu().numpy()
    print(f"  L {L:.17g} oracle {L_ref:.17g}; max |rho diff| {np.abs(new - ref).max():.1e}", flush=True)
    assert abs(L - L_ref) <= 1e-12 * L_ref
    assert np.abs(new - ref).max() <= 1e-12
    assert abs(new.sum() - 0.45 * prob.n_el) <= 1e-9 * prob.n_el


@pytest.mark.parametrize("method", ["fetidp", "tfeti"])
def test_warm_started_design_loop(method):
    prob = workloads.cantilever_tfeti(6, nsub=(4, 2), m=8)
    prob.rho = np.full(prob.n_el, 0.5)
    f = _t(prob.load())
    precond = "dirichlet" if method == "fetidp" else "lumped"
    ctxs = {w: feti.Context(feti.Spec(prob, method=method, scaling="k", krylov="pcg", precond=precond, tol=1e-10,
                                      warm_start=w), _t(prob.rho)) for w in (0, 1)}
    rho = _t(prob.rho)
    for it in range(4):
        print(f"case design loop {method} step {it}", flush=True)
        res = {}
        for w, ctx in ctxs.items():
            c = torch.zeros(1, dtype=torch.float64, device=DEV)
            g = torch.zeros(prob.n_el, dtype=torch.float64, device=DEV)
            u = torch.zeros(prob.n_dof, dtype=torch.float64, device=DEV)
            info = ctx.feti_compliance_and_grad(rho, f, c, g, u)
            res[w] = (info, float(c.cpu()), g, u.cpu().numpy())
        p = workloads.Problem(prob.dim, prob.nel, prob.cuts, rho.cpu().numpy(), Emin=prob.Emin)
        u_star = fem.solve_problem(p)
        c_star = fem.compliance(p.load(), u_star)
        for w in (0, 1):
            info, c, _, u = res[w]
            err = np.linalg.norm(u - u_star) / np.linalg.norm(u_star)
            print(f"  warm {w}: {info['iters']} iterations, u error {err:.1e}, c {c:.12g} (direct {c_star:.12g})",
                  flush=True)
            assert err < 1e-8
            assert abs(c - c_star) <= 1e-9 * abs(c_star)
        if it > 0:   # the oracle, warm-started the same way, saves 2 to 3 of 16 to 17 iterations
            assert res[1][0]["iters"] < res[0][0]["iters"]
        lam = torch.zeros(ctxs[1].sizes["n_lambda"], dtype=torch.float64, device=DEV)
        ctxs[1].feti_get_lambda(lam)
        assert torch.isfinite(lam).all() and torch.count_nonzero(lam) > 0
        new = torch.zeros(prob.n_el, dtype=torch.float64, device=DEV)
        ctxs[1].feti_oc_update(rho, res[1][2], new, 0.5, move=0.02)
        rho = new
    for ctx in ctxs.values():
        ctx.close()
