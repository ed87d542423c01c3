"""Host logic of the C-ABI library checked without a GPU: the library loads, exports every
entry point include/feti.h declares, and its integer topology (interface sizes, lambda
rows with their signs, corner DOFs) equals the oracle's independent construction."""
import os
import re

import numpy as np
import pytest

import workloads
from oracle import topology

feti = pytest.importorskip("paper_2111_11728_amd.feti")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(feti.LIB_PATH):
        pytest.skip("libfeti.so not built (run __graft_entry__.build())")
    return feti.lib()


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    hdr = open(os.path.join(ROOT, "include", "feti.h")).read()
    names = set(re.findall(r"^\s*(?:feti_status|const char\*)\s+(feti_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(L, n), n


def _oracle_rows(prob, method, primal_nodes=None):
    dec = topology.decompose(prob, primal_nodes)
    if method == "tfeti":
        cons = topology.tfeti_constraints(dec)
        rows = [[(s, j, sg) for (s, j, sg) in row] for row in cons.rows]
        return cons, rows, None, dec
    split, cons = topology.fetidp_split(dec)
    rows = [[(s, int(split.r[s][j]), sg) for (s, j, sg) in row] for row in cons.rows]
    return cons, rows, split, dec


CASES = [
    ("c1", lambda: workloads.cantilever_tfeti(0)),
    ("3x3", lambda: workloads.cantilever_tfeti(1, nsub=(3, 3), m=4)),
    ("3d", lambda: workloads.modular_3d(0, nsub=(2, 2, 2), m=3)),
    ("uneven", lambda: workloads.uneven_design(0, 3)),
]


@pytest.mark.parametrize("name,make", CASES)
@pytest.mark.parametrize("method", ["tfeti", "fetidp"])
def test_topology_matches_oracle(name, make, method):
    _lib_or_skip()
    prob = make()
    spec = feti.Spec(prob, method=method)
    sizes = feti.feti_plan_sizes(spec)
    cons, rows, split, dec = _oracle_rows(prob, method)
    assert sizes["n_lambda"] == cons.n_rows
    assert sizes["n_sub"] == prob.n_sub
    # per-subdomain counts
    per = feti.feti_plan_export(spec, 1).reshape(-1, 5)
    nb_or = np.array([b.size for b in cons.bset])
    assert np.array_equal(per[:, 2], nb_or)
    assert np.array_equal(per[:, 0], [sd.n_loc for sd in dec.subs])
    if method == "fetidp":
        assert np.array_equal(per[:, 3], [c.size for c in split.c])
        assert np.array_equal(feti.feti_plan_export(spec, 2), split.corner_dofs)
        assert sizes["n_cg"] == split.corner_dofs.size
    # rows: (subdomain, local DOF, sign) per side, in the same order
    ex = feti.feti_plan_export(spec, 0).reshape(-1, 2, 3)
    assert ex.shape[0] == len(rows)
    for k, row in enumerate(rows):
        got = [tuple(int(v) for v in ex[k, t]) for t in range(2) if ex[k, t, 0] >= 0]
        want = [(s, j, int(sg)) for (s, j, sg) in row]
        assert got == want, (k, got, want)


def test_survey_size_table_c2_c3():
    _lib_or_skip()
    c2 = feti.feti_plan_sizes(feti.Spec(workloads.modular_2d(0), method="fetidp"))
    assert (c2["n_lambda"], c2["n_cg"], c2["nb_max"], c2["nb_min"], c2["sum_nb2"]) == (3224, 76, 248, 124, 1353088)
    c3 = feti.feti_plan_sizes(feti.Spec(workloads.beta_2d(0), method="fetidp"))
    assert (c3["n_lambda"], c3["n_cg"], c3["nb_max"], c3["nb_min"], c3["sum_nb2"]) == (60480, 540, 504, 252, 58042656)
    assert c3["n_groups"] == 64
    t3 = feti.feti_plan_sizes(feti.Spec(workloads.beta_2d(0), method="tfeti"))
    assert (t3["n_lambda"], t3["n_alpha"]) == (65350, 768)
    c5 = feti.feti_plan_sizes(feti.Spec(workloads.modular_3d(0), method="fetidp"))
    assert (c5["n_lambda"], c5["n_cg"], c5["nb_max"], c5["nb_min"], c5["sum_nb2"]) == (77616, 288, 2574, 1320, 258981624)


def test_invalid_inputs_are_rejected():
    _lib_or_skip()
    prob = workloads.cantilever_tfeti(0)
    spec = feti.Spec(prob)
    spec.mesh.nu = 0.7
    with pytest.raises(feti.FetiError) as e:
        feti.feti_plan_sizes(spec)
    assert e.value.status == feti.FETI_EINVAL
    spec = feti.Spec(prob)
    spec.part.nsub[0] = 5      # 32 elements do not split evenly without cuts
    spec.part.cuts[0] = type(spec.part.cuts[0])()
    with pytest.raises(feti.FetiError):
        feti.feti_plan_sizes(spec)


PRIMAL_CASES = [
    ("c2", lambda: workloads.modular_2d(0), 0.2, 3),
    ("c3-block", lambda: workloads.beta_2d_block(1), 0.2, 3),
    ("layered", lambda: workloads.layered_grid(), 0.2, 3),
    ("inclusion", lambda: workloads.inclusion_grid(), 0.5, 2),
    ("uneven", lambda: workloads.uneven_design(0, 3), 0.1, 1),
]


@pytest.mark.parametrize("name,make,theta,cap", PRIMAL_CASES)
def test_adaptive_primal_nodes_match_oracle(name, make, theta, cap):
    """The library's adaptive choice of further primal nodes equals the oracle's (integer output,
    bit-exact), and the FETI-DP topology with the enlarged primal set equals the oracle's."""
    _lib_or_skip()
    prob = make()
    spec = feti.Spec(prob, method="fetidp")
    got = feti.feti_adaptive_primal(spec, theta, cap)
    want = topology.adaptive_primal_nodes(prob, theta, cap)
    assert np.array_equal(got, want)
    assert got.size > 0
    # every chosen node lies strictly inside a shared subdomain edge
    nx = prob.nel[0]
    for nd in got:
        x, y = nd % (nx + 1), nd // (nx + 1)
        assert (x in prob.cuts[0][1:-1]) != (y in prob.cuts[1][1:-1]), nd
    spec = feti.Spec(prob, method="fetidp", primal_nodes=got)
    sizes = feti.feti_plan_sizes(spec)
    cons, rows, split, dec = _oracle_rows(prob, "fetidp", want)
    base = feti.feti_plan_sizes(feti.Spec(prob, method="fetidp"))
    assert sizes["n_cg"] == split.corner_dofs.size == base["n_cg"] + 2 * got.size
    assert sizes["n_lambda"] == cons.n_rows == base["n_lambda"] - 2 * got.size
    assert np.array_equal(feti.feti_plan_export(spec, 2), split.corner_dofs)
    per = feti.feti_plan_export(spec, 1).reshape(-1, 5)
    assert np.array_equal(per[:, 2], [b.size for b in cons.bset])
    assert np.array_equal(per[:, 3], [c.size for c in split.c])
    assert per[:, 3].max() <= 32
    ex = feti.feti_plan_export(spec, 0).reshape(-1, 2, 3)
    for k, row in enumerate(rows):
        got_row = [tuple(int(v) for v in ex[k, t]) for t in range(2) if ex[k, t, 0] >= 0]
        assert got_row == [(s, j, int(sg)) for (s, j, sg) in row], k


def test_primal_nodes_rejected_when_invalid():
    _lib_or_skip()
    prob = workloads.cantilever_tfeti(0)
    for bad in ([5], [0], [10 ** 7]):        # interior node, clamped node, out of range
        with pytest.raises(feti.FetiError) as e:
            feti.feti_plan_sizes(feti.Spec(prob, method="fetidp", primal_nodes=bad))
        assert e.value.status == feti.FETI_EINVAL
    with pytest.raises(feti.FetiError):
        feti.feti_plan_sizes(feti.Spec(prob, method="tfeti", primal_nodes=[8 + 33 * 4]))
    with pytest.raises(ValueError):
        topology.decompose(prob, [5])
