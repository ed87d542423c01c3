"""feti_apply_F_noalloc (the F*Lambda product with its work buffers in the library's fixed
device array) against feti_apply_F, through the C ABI: two calls in a row on two contexts, the
second one smaller, both bit-identical to feti_apply_F on the same inputs; a request whose work
buffers exceed the fixed array is refused with FETI_EINVAL and leaves its output untouched."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
feti = pytest.importorskip("paper_2111_11728_amd.feti")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SCRATCH_BYTES = 16 << 20


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _work_bytes(spec, k):
    """Bytes of the work buffers of one F*Lambda with k columns (the header's formula)."""
    per_sub = feti.feti_plan_export(spec, 1).reshape(-1, 5)
    nb_tot, nc_tot = int(per_sub[:, 2].sum()), int(per_sub[:, 3].sum())
    n_cg = feti.feti_plan_sizes(spec)["n_cg"]
    up = lambda b: (b + 255) // 256 * 256  # noqa: E731
    return up(8 * max(1, nb_tot) * k) + up(8 * max(1, nc_tot) * k) + 2 * up(8 * max(1, n_cg) * k)


def _case(prob, k, product_precision, seed, **kw):
    spec = feti.Spec(prob, **kw)
    assert _work_bytes(spec, k) <= SCRATCH_BYTES
    ctx = feti.Context(spec, _t(prob.rho))
    n = ctx.sizes["n_lambda"]
    L = _t(np.random.default_rng(seed).standard_normal((n, k)))
    Q_ref = torch.zeros((n, k), dtype=torch.float64, device=DEV)
    Q = torch.full((n, k), np.nan, dtype=torch.float64, device=DEV)
    ctx.feti_apply_F(k, product_precision, L, Q_ref)
    ctx.feti_apply_F_noalloc(k, product_precision, L, Q)
    torch.cuda.synchronize()
    ctx.close()
    return Q, Q_ref


def test_apply_F_noalloc_matches_apply_F_twice():
    print("case no-alloc F*Lambda: 8x4 modular design of 16^2 (FETI-DP, hybrid FP32), k = 64", flush=True)
    big = workloads.modular_2d(3, nsub=(8, 4), m=16)
    Q, Q_ref = _case(big, 64, "fp32", 5, method="fetidp", scaling="k", krylov="sfeti", precision="fp32")
    assert torch.isfinite(Q).all()
    assert torch.equal(Q, Q_ref)
    print("case no-alloc F*Lambda: 4x2 cantilever of 8^2 (TFETI, FP64), k = 5", flush=True)
    small = workloads.cantilever_tfeti(1)
    Q, Q_ref = _case(small, 5, "fp64", 6, method="tfeti", scaling="mult", precond="lumped")
    assert torch.isfinite(Q).all()
    assert torch.equal(Q, Q_ref)
    print("case no-alloc F*Lambda: 4x2 cantilever of 8^2 (FETI-DP, FP64), k = 1", flush=True)
    Q, Q_ref = _case(small, 1, "fp64", 7, method="fetidp", scaling="k")
    assert torch.equal(Q, Q_ref)


def test_apply_F_noalloc_refuses_oversized_workspace():
    # 3D, 4x4x4 subdomains of 7^3 elements: the 64-column work buffers exceed 16 MiB
    prob = workloads.modular_3d(2, nsub=(4, 4, 4), m=7)
    spec = feti.Spec(prob, method="fetidp", scaling="k")
    assert _work_bytes(spec, 64) > SCRATCH_BYTES
    assert _work_bytes(spec, 16) <= SCRATCH_BYTES
    print("case no-alloc F*Lambda: 3D 4x4x4 of 7^3, k = 64 (refused) and k = 16", flush=True)
    ctx = feti.Context(spec, _t(prob.rho))
    n = ctx.sizes["n_lambda"]
    L = _t(np.random.default_rng(8).standard_normal((n, 64)))
    Q = torch.zeros((n, 64), dtype=torch.float64, device=DEV)
    with pytest.raises(feti.FetiError) as ei:
        ctx.feti_apply_F_noalloc(64, "fp64", L, Q)
    assert ei.value.status == feti.FETI_EINVAL
    torch.cuda.synchronize()
    assert torch.count_nonzero(Q) == 0
    L16 = L[:, :16].contiguous()
    Q16 = torch.zeros((n, 16), dtype=torch.float64, device=DEV)
    Q16_ref = torch.zeros((n, 16), dtype=torch.float64, device=DEV)
    ctx.feti_apply_F(16, "fp64", L16, Q16_ref)
    ctx.feti_apply_F_noalloc(16, "fp64", L16, Q16)
    torch.cuda.synchronize()
    ctx.close()
    assert torch.equal(Q16, Q16_ref)
