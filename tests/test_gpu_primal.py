"""FETI-DP with an enlarged primal set (Sec. 2.2 with primal nodes beyond the corners, the
adaptive choice of the paper's Sec. 6, item i) on the HIP path, against the oracle run with the
oracle's own choice of the same nodes (tests/test_host_plan.py checks that both choices agree).

Per problem and Krylov method (PCG, simultaneous directions), Dirichlet preconditioner,
k-scaling, tol 1e-8: u against the global direct solution within 10x the oracle's own distance;
the iteration count within the oracle's round-off spread (its dense-F run) or 1; and, on the
layered grid and the inclusion grid, no more iterations than with the corners alone."""
import numpy as np
import pytest

import workloads
from oracle import fem, topology
from oracle import feti as ofeti
from oracle import krylov as okrylov

torch = pytest.importorskip("torch")
feti = pytest.importorskip("paper_2111_11728_amd.feti")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-8

CASES = {
    "layered_grid": workloads.layered_grid,
    "inclusion_grid": workloads.inclusion_grid,
    "modular_4x4_of_16": lambda: workloads.modular_2d(1, nsub=(4, 4), m=16),
}


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


class _DenseF:
    def __init__(self, op):
        self.op = op
        F = op.apply_F(np.eye(op.n_lambda))
        self.F = 0.5 * (F + F.T)
        self.n_lambda = op.n_lambda
        self.d = op.d

    def apply_F(self, L):
        return self.F @ L

    def project(self, Y):
        return self.op.project(Y)

    def lambda0(self):
        return self.op.lambda0()

    def precondition(self, r, one_column=False):
        return self.op.precondition(r, one_column)


def _gpu(prob, kr, nodes):
    spec = feti.Spec(prob, method="fetidp", scaling="k", krylov=kr, precond="dirichlet", tol=TOL,
                     primal_nodes=nodes)
    ctx = feti.Context(spec, _t(prob.rho))
    u = torch.zeros(prob.n_dof, dtype=torch.float64, device=DEV)
    info = ctx.feti_solve(_t(prob.load()), u, allow_noconv=True)
    n_cg = ctx.sizes["n_cg"]
    ctx.close()
    return info, u.cpu().numpy(), n_cg


@pytest.mark.parametrize("kr", ["pcg", "sfeti"])
@pytest.mark.parametrize("name", list(CASES))
def test_enlarged_primal_set_against_oracle(name, kr):
    prob = CASES[name]()
    nodes_lib = feti.feti_adaptive_primal(feti.Spec(prob, method="fetidp"))
    nodes_orc = topology.adaptive_primal_nodes(prob)
    assert np.array_equal(nodes_lib, nodes_orc) and nodes_lib.size > 0
    u_star = fem.solve_problem(prob)
    op = ofeti.FETIDP(prob, "dirichlet", "k", primal_nodes=nodes_orc)
    res = okrylov.solve(op, kr, tol=TOL)
    res_d = okrylov.solve(_DenseF(op), kr, tol=TOL)
    u_o, _ = op.recover(res.lam)
    err_o = np.linalg.norm(u_o - u_star) / np.linalg.norm(u_star)
    print(f"case primal {name} {kr}: {nodes_lib.size} further primal nodes", flush=True)
    info, u, n_cg = _gpu(prob, kr, nodes_lib)
    err = np.linalg.norm(u - u_star) / np.linalg.norm(u_star)
    info0, _, n_cg0 = _gpu(prob, kr, None)
    print(f"  gpu {info['iters']} iterations (corners only {info0['iters']}), oracle {res.iters} "
          f"(dense F {res_d.iters}); n_cg {n_cg} (corners {n_cg0}); u error gpu {err:.1e}, oracle {err_o:.1e}",
          flush=True)
    assert n_cg == n_cg0 + 2 * nodes_lib.size == op.n_cg
    assert (info["status"] == feti.FETI_OK) == res.converged
    spread = abs(res.iters - res_d.iters)
    # plain PCG loses orthogonality here: twice the measured round-off spread, at least 2
    assert abs(info["iters"] - res.iters) <= (max(2, 2 * spread) if kr == "pcg" else max(1, spread))
    if res.converged:
        assert err <= 10.0 * err_o + 1e-12
    if name != "modular_4x4_of_16":
        assert info["iters"] <= info0["iters"]
