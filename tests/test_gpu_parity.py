"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: FP64 local operators and F*Lambda agree to 1e-11 relative (rounding order
only); FP32 F*Lambda to 2e-6 and split-BF16 (three products) to 5e-5 relative in the
Frobenius norm (FP32 accumulation over n_b <= 504 terms of FP32-rounded / BF16-split
operands); solutions: FP64 path <= 1e-8 relative to the oracle, mixed precision <= 1e-6,
plain PCG iteration counts within 1 of the oracle's.
"""
import numpy as np
import pytest

import workloads
from oracle import fem
from oracle import feti as ofeti
from oracle import krylov as okrylov

torch = pytest.importorskip("torch")
feti = pytest.importorskip("paper_2111_11728_amd.feti")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def _ctx(prob, **kw):
    spec = feti.Spec(prob, **kw)
    return feti.Context(spec, _t(prob.rho))


SMALL = {
    "c1": lambda: workloads.cantilever_tfeti(0),
    "3x3": lambda: workloads.cantilever_tfeti(2, nsub=(3, 3), m=5),
    "uneven": lambda: workloads.uneven_design(1, 0),
    "3d": lambda: workloads.modular_3d(1, nsub=(2, 2, 2), m=3),
}


@pytest.fixture(scope="module")
def oracle_cache():
    return {}


def _oracle(cache, name, method, precond, scaling):
    key = (name, method, precond, scaling)
    if key not in cache:
        prob = SMALL[name]()
        cls = ofeti.TFETI if method == "tfeti" else ofeti.FETIDP
        cache[key] = (prob, cls(prob, precond, scaling))
    return cache[key]


@pytest.mark.parametrize("name", ["c1", "3x3", "uneven", "3d"])
@pytest.mark.parametrize("precond", ["dirichlet", "lumped"])
def test_fetidp_local_operators(oracle_cache, name, precond):
    prob, op = _oracle(oracle_cache, name, "fetidp", precond, "k")
    print(f"case {name} fetidp {precond}", flush=True)
    ctx = _ctx(prob, method="fetidp", scaling="k", precond=precond)
    for s in range(prob.n_sub):
        Fs = ctx.feti_get_local(s, 0)
        assert _rel(Fs, op.F_local[s]) < 1e-11, s
        assert _rel(ctx.feti_get_local(s, 1), op.S[s]) < 1e-12, s
        if op.Frc[s].size:
            assert _rel(ctx.feti_get_local(s, 2), op.Frc[s]) < 1e-11, s
            assert _rel(ctx.feti_get_local(s, 3), op.Kcc_bar[s]) < 1e-11, s
    if op.n_cg:
        assert _rel(ctx.feti_get_local(0, 5), op.Kcc_glob) < 1e-11
    w = ctx.feti_get_local(0, 4)
    for s in range(prob.n_sub):
        ex = feti.feti_plan_export(ctx.spec, 0).reshape(-1, 2, 3)
        break
    wo = np.zeros((op.n_lambda, 2))
    for r in range(op.n_lambda):
        for t in range(2):
            s = ex[r, t, 0]
            if s >= 0:
                wo[r, t] = op.w[s][r]
    assert np.abs(w - wo).max() < 1e-14
    ctx.close()


@pytest.mark.parametrize("name", ["c1", "3x3", "uneven", "3d"])
@pytest.mark.parametrize("method", ["fetidp", "tfeti"])
@pytest.mark.parametrize("k", [1, 7, 64])
def test_apply_F_fp64(oracle_cache, name, method, k):
    precond = "dirichlet" if method == "fetidp" else "lumped"
    prob, op = _oracle(oracle_cache, name, method, precond, "mult")
    print(f"case {name} {method} k={k}", flush=True)
    ctx = _ctx(prob, method=method, scaling="mult", precond=precond)
    n = op.n_lambda
    rng = np.random.default_rng(k)
    L = rng.standard_normal((n, k))
    Lt = _t(L)
    if method == "tfeti":
        ctx.feti_project(k, Lt)
        PL = op.project(L)
        assert _rel(Lt.cpu().numpy(), PL) < 1e-12
    Q = torch.zeros_like(Lt)
    ctx.feti_apply_F(k, "fp64", Lt, Q)
    if method == "tfeti":
        ctx.feti_project(k, Q)
        ref = op.project(op.apply_F(op.project(L)))
    else:
        ref = op.apply_F(L)
    assert _rel(Q.cpu().numpy(), ref) < 1e-11
    ctx.close()


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-6), ("bf16x3", 5e-5)])
@pytest.mark.parametrize("name", ["c1", "uneven", "3d"])
def test_apply_F_mixed(oracle_cache, name, precision, tol):
    prob, op = _oracle(oracle_cache, name, "fetidp", "dirichlet", "mult")
    print(f"case {name} {precision}", flush=True)
    ctx = _ctx(prob, method="fetidp", scaling="mult")
    n = op.n_lambda
    L = np.random.default_rng(3).standard_normal((n, 64))
    Q = torch.zeros((n, 64), dtype=torch.float64, device=DEV)
    ctx.feti_apply_F(64, precision, _t(L), Q)
    assert _rel(Q.cpu().numpy(), op.apply_F(L)) < tol
    ctx.close()


@pytest.mark.parametrize("name", ["c1", "3x3", "3d"])
@pytest.mark.parametrize("method", ["fetidp", "tfeti"])
def test_preconditioner_and_rhs(oracle_cache, name, method):
    precond = "dirichlet"
    prob, op = _oracle(oracle_cache, name, method, precond, "k")
    print(f"case {name} {method}", flush=True)
    ctx = _ctx(prob, method=method, scaling="k", precond=precond)
    n = op.n_lambda
    r = np.random.default_rng(5).standard_normal(n)
    Z1 = torch.zeros(n, dtype=torch.float64, device=DEV)
    ctx.feti_apply_precond(_t(r), Z1, 1)
    assert _rel(Z1.cpu().numpy(), op.precondition(r, one_column=True)[:, 0]) < 1e-12
    kz = ctx.sizes["n_groups"]
    Zk = torch.zeros((n, kz), dtype=torch.float64, device=DEV)
    ctx.feti_apply_precond(_t(r), Zk, 0)
    assert _rel(Zk.cpu().numpy(), op.precondition(r)) < 1e-12
    d = torch.zeros(n, dtype=torch.float64, device=DEV)
    l0 = torch.zeros(n, dtype=torch.float64, device=DEV)
    ctx.feti_rhs(_t(prob.load()), d, l0)
    lam0 = op.lambda0()
    assert np.abs(l0.cpu().numpy() - lam0).max() <= 1e-11 * max(1.0, np.abs(lam0).max())
    if method == "fetidp":
        assert _rel(d.cpu().numpy(), op.d) < 1e-11
    else:
        # generalised-inverse independent: P(d - F lambda0)
        Q = torch.zeros((n, 1), dtype=torch.float64, device=DEV)
        ctx.feti_apply_F(1, "fp64", _t(lam0[:, None]), Q)
        rg = _t(d.cpu().numpy() - Q.cpu().numpy()[:, 0])[:, None].contiguous()
        ctx.feti_project(1, rg)
        ro = op.project((op.d - op.apply_F(lam0[:, None])[:, 0])[:, None])[:, 0]
        assert _rel(rg.cpu().numpy()[:, 0], ro) < 1e-10
    ctx.close()


@pytest.mark.parametrize("method", ["tfeti", "fetidp"])
@pytest.mark.parametrize("scaling", ["mult", "k"])
@pytest.mark.parametrize("kr", ["pcg", "fo", "sfeti"])
def test_twelve_variants_c1(method, scaling, kr):
    """Every variant of the paper's comparison on the 4x2 cantilever (FP64)."""
    prob = workloads.cantilever_tfeti(0)
    precond = "lumped" if method == "tfeti" else "dirichlet"
    print(f"case c1 {method} {scaling} {kr}", flush=True)
    cls = ofeti.TFETI if method == "tfeti" else ofeti.FETIDP
    op = cls(prob, precond, scaling)
    res = okrylov.solve(op, kr, tol=1e-10)
    u_ref, _ = op.recover(res.lam)
    ctx = _ctx(prob, method=method, scaling=scaling, krylov=kr, precond=precond, tol=1e-10)
    u = torch.zeros(prob.n_dof, dtype=torch.float64, device=DEV)
    info = ctx.feti_solve(_t(prob.load()), u)
    assert _rel(u.cpu().numpy(), u_ref) < 1e-8
    assert _rel(u.cpu().numpy(), fem.solve_problem(prob)) < 1e-8
    if kr == "pcg":
        assert abs(info["iters"] - res.iters) <= 1
        assert np.allclose(info["history"][:5], res.history[:5], rtol=1e-8)
    else:
        assert abs(info["iters"] - res.iters) <= 2
    ctx.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mixed_precision_solve(precision):
    prob = workloads.cantilever_tfeti(0, nsub=(4, 4), m=8)
    print(f"case mixed {precision}", flush=True)
    ctx = _ctx(prob, method="fetidp", scaling="k", krylov="sfeti", precision=precision, tol=1e-8)
    u = torch.zeros(prob.n_dof, dtype=torch.float64, device=DEV)
    info = ctx.feti_solve(_t(prob.load()), u)
    assert info["true_rel_res"] <= 1e-8
    assert _rel(u.cpu().numpy(), fem.solve_problem(prob)) < 1e-6
    ctx.close()


def test_c2_sfeti_fetidp():
    """Modular 8x4 design of 32x32 modules: S-FETI-DP with k-scaling, FP64 and FP32."""
    prob = workloads.modular_2d(0)
    op = ofeti.FETIDP(prob, "dirichlet", "k")
    res = okrylov.solve(op, "sfeti", tol=1e-8)
    u_ref, _ = op.recover(res.lam)
    for precision in ["fp64", "fp32"]:
        print(f"case c2 sfeti {precision}", flush=True)
        ctx = _ctx(prob, method="fetidp", scaling="k", krylov="sfeti", precision=precision, tol=1e-8)
        u = torch.zeros(prob.n_dof, dtype=torch.float64, device=DEV)
        info = ctx.feti_solve(_t(prob.load()), u)
        err = _rel(u.cpu().numpy(), u_ref)
        assert err < (1e-8 if precision == "fp64" else 1e-6), err
        if precision == "fp64":
            assert abs(info["iters"] - res.iters) <= 2
        ctx.close()


def test_compliance_gradient_small():
    prob = workloads.cantilever_tfeti(3, nsub=(2, 2), m=4)
    print("case compliance", flush=True)
    ctx = _ctx(prob, method="fetidp", scaling="k", krylov="sfeti", tol=1e-12)
    c = torch.zeros(1, dtype=torch.float64, device=DEV)
    g = torch.zeros(prob.n_el, dtype=torch.float64, device=DEV)
    u = torch.zeros(prob.n_dof, dtype=torch.float64, device=DEV)
    ctx.feti_compliance_and_grad(_t(prob.rho), _t(prob.load()), c, g, u)
    u_ref = fem.solve_problem(prob)
    assert float(c.cpu()) == pytest.approx(fem.compliance(prob.load(), u_ref), rel=1e-9)
    assert _rel(g.cpu().numpy(), fem.compliance_gradient(prob, u_ref)) < 1e-8
    ctx.close()
