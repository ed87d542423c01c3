"""Pins of the oracle's dual operators and Krylov iterations against the global
direct solve, the explicit saddle-point systems (Sec. 2.1 Eq. 6, Sec. 2.2 Eq. 11),
invariants of the projected iteration, scipy's CG on the same explicit operator,
and brute force for the rank-revealing Cholesky (no GPU)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads
from oracle import fem, feti, krylov, topology


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def c1():
    p = workloads.cantilever_tfeti(0)
    return p, fem.solve_problem(p)


@pytest.mark.parametrize("method", ["tfeti", "fetidp"])
@pytest.mark.parametrize("scaling", ["mult", "k"])
@pytest.mark.parametrize("kr", ["pcg", "fo", "sfeti"])
def test_twelve_variants_reach_direct_solution(c1, method, scaling, kr):
    """Every variant of Sec. 4 (method x scaling x Krylov) converges to u* = K^{-1} f."""
    prob, ustar = c1
    op = feti.TFETI(prob, "lumped", scaling) if method == "tfeti" else feti.FETIDP(prob, "dirichlet", scaling)
    res = krylov.solve(op, kr, tol=1e-12)
    assert res.converged
    u, _ = op.recover(res.lam)
    assert _rel(u, ustar) < 1e-8


def test_tfeti_operator_is_pseudo_inverse_block(c1):
    """F = B K^+ B^T with K^+ from an SVD pseudo-inverse; F symmetric PSD; PFP SPD on range P."""
    prob, _ = c1
    op = feti.TFETI(prob)
    n = op.n_lambda
    F = op.apply_F(np.eye(n))
    Fref = sum((op.cons.B[s] @ np.linalg.pinv(op.K[s].toarray(), rcond=1e-13, hermitian=True)
                @ op.cons.B[s].T.toarray()) for s in range(len(op.K)))
    assert np.abs(F - Fref).max() < 1e-9 * np.abs(F).max()
    assert np.allclose(F, F.T, atol=1e-12 * np.abs(F).max())
    assert np.linalg.eigvalsh(F).min() > -1e-12 * np.abs(F).max()
    P = op.project(np.eye(n))
    PFP = P @ F @ P
    ev = np.linalg.eigvalsh(PFP)
    rankP = int(round(np.trace(P)))
    assert rankP == n - op.G.shape[0]
    # PFP has exactly n - rank(P) (near-)zero eigenvalues... plus those of B's redundancy
    assert ev.min() > -1e-12 * ev.max()


def test_tfeti_saddle_point_system(c1):
    """The KKT system [K B^T; B 0][u; lambda] = [f; c] (Eq. 6) has the torn direct solution as u."""
    prob, ustar = c1
    op = feti.TFETI(prob)
    K = sp.block_diag(op.K).toarray()
    B = sp.hstack(op.cons.B).toarray()
    f = np.concatenate(op.fs)
    A = np.block([[K, B.T], [B, np.zeros((B.shape[0], B.shape[0]))]])
    rhs = np.concatenate([f, np.zeros(B.shape[0])])
    sol = np.linalg.lstsq(A, rhs, rcond=1e-12)[0]
    u_t = sol[:K.shape[0]]
    off = 0
    for sd in op.dec.subs:
        assert np.abs(u_t[off:off + sd.n_loc] - ustar[sd.dofs]).max() < 1e-8 * np.abs(ustar).max()
        off += sd.n_loc


def test_tfeti_generalized_inverse_invariance(c1):
    """PFP, P(d - F lambda) for feasible lambda and the PCG iterates do not depend on which generalised inverse of K^s is
    used: replace K^+ by the inverse with three DOFs fixed (not Moore-Penrose)."""
    prob, ustar = c1
    op = feti.TFETI(prob)
    ref = krylov.pcg(op, tol=1e-12)
    op2 = feti.TFETI(prob)
    for s, Ks in enumerate(op2.K):
        A = Ks.toarray()
        keep = np.setdiff1d(np.arange(A.shape[0]), [0, 1, 3])   # node 0 (u,v) and node 1 (v)
        Kg = np.zeros_like(A)
        Kg[np.ix_(keep, keep)] = np.linalg.inv(A[np.ix_(keep, keep)])
        assert np.abs(A @ Kg @ A - A).max() < 1e-10 * np.abs(A).max()
        op2.Kdag[s] = Kg
        b = op2.b_local[s]
        op2.F_local[s] = Kg[b][:, b]
    op2.d = sum(op2.cons.B[s] @ (op2.Kdag[s] @ op2.fs[s]) for s in range(len(op2.K)))
    n = op.n_lambda
    P = op.project(np.eye(n))
    assert np.abs(P @ op.apply_F(P) - P @ op2.apply_F(P)).max() < 1e-9 * np.abs(op.apply_F(P)).max()
    # the projected residual of any feasible lambda (G lambda = e) is the same
    lam0 = op.lambda0()
    r_a = P @ (op.d - op.apply_F(lam0[:, None])[:, 0])
    r_b = P @ (op2.d - op2.apply_F(lam0[:, None])[:, 0])
    assert np.abs(r_a - r_b).max() < 1e-9 * np.abs(r_a).max()
    res2 = krylov.pcg(op2, tol=1e-12)
    assert abs(res2.iters - ref.iters) <= 1
    u2, _ = op2.recover(res2.lam)
    assert _rel(u2, ustar) < 1e-8


def test_fetidp_condensed_operator_is_kkt_schur(c1):
    """F_DP = Schur complement onto lambda of the primal 3x3 system (Eq. 11), and
    d_DP the matching right-hand side."""
    prob, _ = c1
    op = feti.FETIDP(prob)
    n = op.n_lambda
    FDP = op.apply_F(np.eye(n))
    # global blocks of Eq. (11): unknowns [u_c (global corners), u_r (all subdomains)]
    nsub = len(op.K)
    Kcc = np.zeros((op.n_cg, op.n_cg))
    blocks_rr, Kcr_cols, Br_cols, fr = [], [], [], []
    fc = np.zeros(op.n_cg)
    for s in range(nsub):
        r, c = op.split.r[s], op.split.c[s]
        Ks = op.K[s].toarray()
        Bc = op.split.Bc[s].toarray()
        Kcc += Bc.T @ Ks[np.ix_(c, c)] @ Bc
        blocks_rr.append(Ks[np.ix_(r, r)])
        Kcr_cols.append(Bc.T @ Ks[np.ix_(c, r)])
        Br_cols.append(op.cons.B[s].toarray())
        fr.append(op.fs[s][r])
        fc += Bc.T @ op.fs[s][c]
    Krr = sla.block_diag(*blocks_rr)
    Kcr = np.hstack(Kcr_cols)
    Br = np.hstack(Br_cols)
    A = np.block([[Kcc, Kcr], [Kcr.T, Krr]])
    C = np.hstack([np.zeros((n, op.n_cg)), Br])
    S = C @ np.linalg.solve(A, C.T)
    assert np.abs(FDP - S).max() < 1e-8 * np.abs(S).max()
    dref = C @ np.linalg.solve(A, np.concatenate([fc, np.concatenate(fr)]))
    assert np.abs(op.d - dref).max() < 1e-8 * np.abs(dref).max()


def test_fetidp_continuity_of_recovered_copies(c1):
    prob, _ = c1
    op = feti.FETIDP(prob, "dirichlet", "k")
    res = krylov.pcg(op, tol=1e-12)
    _, us = op.recover(res.lam)
    jump = sum(op.cons.B[s] @ us[s][op.split.r[s]] for s in range(len(us)))
    assert np.abs(jump).max() < 1e-9 * max(np.abs(u).max() for u in us)


def test_tfeti_feasibility_at_every_iterate(c1):
    """G lambda = e, i.e. R^T (f - B^T lambda) = 0 per subdomain, at every PCG iterate."""
    prob, _ = c1
    op = feti.TFETI(prob)
    for it in [1, 3, 7]:
        res = krylov.pcg(op, tol=0.0, max_it=it)
        assert np.abs(op.G @ res.lam - op.e).max() < 1e-12 * np.abs(op.e).max()
        for s in range(len(op.K)):
            assert np.abs(op.R[s].T @ (op.fs[s] - op.cons.B[s].T @ res.lam)).max() < 1e-12


def test_pcg_matches_scipy_cg_iterates():
    """The oracle's PCG on F_DP with the Dirichlet preconditioner produces the same iterates
    as scipy's CG on the explicit matrices (same textbook recurrence)."""
    prob = workloads.cantilever_tfeti(1, nsub=(3, 2), m=4)
    op = feti.FETIDP(prob, "dirichlet", "k")
    n = op.n_lambda
    F = op.apply_F(np.eye(n))
    M = op.precondition(np.eye(n)[:, 0], one_column=True)  # warm the code path
    M = np.column_stack([op.precondition(e, one_column=True)[:, 0] for e in np.eye(n)])
    iters = []
    spla.cg(F, op.d, x0=np.zeros(n), M=M, rtol=1e-30, maxiter=6, callback=lambda x: iters.append(x.copy()))
    for k in [1, 3, 6]:
        res = krylov.pcg(op, tol=0.0, max_it=k)
        assert _rel(res.lam, iters[k - 1]) < 1e-10


def test_fo_equals_pcg_initially_and_sfeti_one_group_is_fo(c1):
    prob, _ = c1
    op = feti.FETIDP(prob, "dirichlet", "mult")
    for k in [1, 2, 4]:
        a = krylov.pcg(op, tol=0.0, max_it=k)
        b = krylov.simultaneous(op, tol=0.0, max_it=k, one_group=True)
        assert _rel(b.lam, a.lam) < 1e-10
        assert np.allclose(a.history, b.history, rtol=1e-9)


def test_sfeti_directions_are_F_orthonormal(c1):
    """After the normalisation of Algorithm 1, W^T F W = I for the kept directions and
    successive blocks are F-orthogonal."""
    prob, _ = c1
    op = feti.FETIDP(prob, "dirichlet", "k")
    lam0 = op.lambda0()
    r = op.d - op.apply_F(lam0[:, None])[:, 0]
    W = op.precondition(r)
    Q = op.apply_F(W)
    T, rank = krylov.pivoted_cholesky(Q.T @ W)
    W1 = W @ T
    assert np.allclose(W1.T @ op.apply_F(W1), np.eye(rank), atol=1e-10)
    # second block orthogonalised against the first
    Q1 = op.apply_F(W1)
    r1 = r - Q1 @ (W1.T @ r)
    W2 = op.precondition(r1)
    W2 = W2 - W1 @ (Q1.T @ W2)
    assert np.abs(W1.T @ op.apply_F(W2)).max() < 1e-10 * np.abs(op.apply_F(W2)).max()
    # w = W 1 recovers the classical direction (Sec. 3.3)
    assert np.allclose(op.precondition(r).sum(axis=1), op.precondition(r, one_column=True)[:, 0])


def test_pivoted_cholesky_brute_force():
    rng = np.random.default_rng(0)
    # full rank: T^T D T = I, rank k
    A = rng.standard_normal((30, 6))
    D = A.T @ A
    T, rank = krylov.pivoted_cholesky(D)
    assert rank == 6 and np.allclose(T.T @ D @ T, np.eye(6), atol=1e-12)
    # duplicated and scaled columns: rank of the independent set
    V = rng.standard_normal((40, 4))
    Vd = np.column_stack([V, 3.0 * V[:, 1], V[:, 0] + V[:, 2], np.zeros(40)])
    D = Vd.T @ Vd
    T, rank = krylov.pivoted_cholesky(D)
    assert rank == 4
    assert np.allclose(T.T @ D @ T, np.eye(4), atol=1e-10)
    assert np.abs(T[6]).max() == 0.0               # the zero column is never used
    # a tiny but independent direction survives thanks to the Jacobi scaling
    Vs = np.column_stack([V[:, :3], 1e-7 * V[:, 3]])
    T, rank = krylov.pivoted_cholesky(Vs.T @ Vs)
    assert rank == 4
    # pivot order on the scaled matrix: first pivot is column 0 (all scaled diagonals are 1)
    D = np.diag([4.0, 9.0, 1.0])
    T, rank = krylov.pivoted_cholesky(D)
    assert rank == 3 and np.allclose(T, np.diag([0.5, 1 / 3, 1.0]))
    # k = 1 is the normalisation of FO
    T, rank = krylov.pivoted_cholesky(np.array([[4.0]]))
    assert rank == 1 and T[0, 0] == 0.5


def test_load_split_invariance():
    """u does not depend on which subdomain carries a load on a shared node."""
    prob = workloads.cantilever_tfeti(0, nsub=(2, 2), m=4)
    op = feti.FETIDP(prob, "dirichlet", "k")
    res = krylov.pcg(op, tol=1e-13)
    u1, _ = op.recover(res.lam)
    # move the right-mid load (node on the horizontal interface) to the upper subdomain
    g = int(np.nonzero(op.f)[0][0])
    owners = [sd.index for sd in op.dec.subs if g in op.dec.g2l[sd.index]]
    assert len(owners) == 2
    for s in owners:
        op.fs[s][:] = 0.0
    op.fs[owners[1]][op.dec.g2l[owners[1]][g]] = op.f[g]
    op2 = feti.FETIDP.__new__(feti.FETIDP)
    op2.__dict__.update(op.__dict__)
    # rebuild d_r and fbar_c with the moved load
    d_r = np.zeros(op.n_lambda)
    fbar = np.zeros(op.n_cg)
    for s in range(len(op.K)):
        r, c = op.split.r[s], op.split.c[s]
        xr = op.lu[s].solve(op.fs[s][r])
        d_r += op.cons.B[s] @ xr
        fbar += op.split.Bc[s].T @ (op.fs[s][c] - op.Krc[s].T @ xr)
    op2.d_r, op2.fbar_c = d_r, fbar
    op2.d = d_r - op2.apply_Frc(op2.coarse_solve(fbar[:, None]))[:, 0]
    res2 = krylov.pcg(op2, tol=1e-13)
    u2, _ = op2.recover(res2.lam)
    assert _rel(u2, u1) < 1e-9


def test_all_primal_degenerate_case():
    """Every interface node primal: FETI-DP has no multipliers and is a primal Schur
    method; u equals the direct solution exactly (to round-off)."""
    prob = workloads.cantilever_tfeti(4, nsub=(2, 1), m=1)
    op = feti.FETIDP(prob, "dirichlet", "k")
    assert op.n_lambda == 0
    u, _ = op.recover(np.zeros(0))
    assert _rel(u, fem.solve_problem(prob)) < 1e-12


def test_3d_fetidp_small():
    prob = workloads.modular_3d(0, nsub=(2, 2, 2), m=3)
    op = feti.FETIDP(prob, "dirichlet", "k")
    res = krylov.solve(op, "sfeti", tol=1e-12)
    u, _ = op.recover(res.lam)
    assert res.converged and _rel(u, fem.solve_problem(prob)) < 1e-8


def test_fetidp_local_against_dense_inverse():
    """One subdomain's F_s, F_rc^s and Kbar_cc^s (Sec. 2.2, Eq. 11-12) against their definitions
    written with a dense inverse of K_rr (no LU, no right-hand-side blocking): F_s = (K_rr^{-1})_bb,
    F_rc^s = (K_rr^{-1} K_rc)_b, Kbar_cc^s = K_cc - K_rc^T K_rr^{-1} K_rc; plus symmetry and
    positive definiteness of F_s."""
    prob = workloads.cantilever_tfeti(3, nsub=(3, 2), m=4)
    dec = topology.decompose(prob)
    split, cons = topology.fetidp_split(dec)
    E = fem.simp_modulus(prob.rho, prob.p, prob.E0, prob.Emin)
    K0 = fem.element_stiffness(prob.dim, prob.nu)
    for s in range(len(dec.subs)):
        Ks = feti.subdomain_stiffness(prob, dec.subs[s], E, K0).toarray()
        r, c, bpos = split.r[s], split.c[s], cons.bset[s]
        Fs, Frc, Kcc_bar, _, _ = feti.fetidp_local(sp.csr_matrix(Ks), r, c, bpos)
        Kinv = np.linalg.inv(Ks[np.ix_(r, r)])
        Krc = Ks[np.ix_(r, c)]
        assert np.allclose(Fs, Kinv[np.ix_(bpos, bpos)], rtol=1e-10, atol=1e-12 * np.abs(Kinv).max())
        if c.size:
            assert np.allclose(Frc, (Kinv @ Krc)[bpos], rtol=1e-10, atol=1e-12 * np.abs(Kinv @ Krc).max())
            ref = Ks[np.ix_(c, c)] - Krc.T @ Kinv @ Krc
            assert np.allclose(Kcc_bar, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())
        assert np.allclose(Fs, Fs.T, atol=1e-12 * np.abs(Fs).max())
        assert np.linalg.eigvalsh(0.5 * (Fs + Fs.T)).min() > 0.0


@pytest.mark.parametrize("method", ["tfeti", "fetidp"])
def test_dirichlet_schur_is_harmonic_extension_energy(method):
    """The Dirichlet block S^s of the preconditioner (Sec. 3.1, Eq. 13) against the energy
    characterisation of a Schur complement, written without its block formula: for a trace x_b on
    the interface, the least strain energy x^T K_A x over all interior completions x_i is x_b^T S x_b
    (K_A = K^s on the active DOFs: all local DOFs in TFETI, the remainder set r in FETI-DP, Sec. 2.2).
    The minimiser (the harmonic extension) solves K_ii x_i = -K_ib x_b; it is computed here with a
    dense solve, the energy with the full active matrix, and S_ref = X^T K_A X with the unit traces
    as columns. Any other completion has more energy. TFETI: rigid-body traces carry no energy,
    S R_b = 0 on every (floating) subdomain. Heterogeneous densities (U(0, 1), contrast 1e-6)."""
    prob = workloads.cantilever_tfeti(7, nsub=(3, 2), m=4)
    op = feti.TFETI(prob, "dirichlet", "mult") if method == "tfeti" else feti.FETIDP(prob, "dirichlet", "mult")
    rng = np.random.default_rng(3)
    for s, sd in enumerate(op.dec.subs):
        K = op.K[s].toarray()
        active = np.arange(sd.n_loc) if method == "tfeti" else op.split.r[s]
        b = np.asarray(op.b_local[s])
        i = np.setdiff1d(active, b)
        X = np.zeros((sd.n_loc, b.size))
        X[b, np.arange(b.size)] = 1.0
        X[i] = np.linalg.solve(K[np.ix_(i, i)], -K[np.ix_(i, b)])
        S_ref = X.T @ K @ X
        S = op.S[s]
        assert np.abs(S - S_ref).max() <= 1e-10 * np.abs(S_ref).max(), s
        # minimality: a perturbed interior raises the energy of a random trace
        xb = rng.standard_normal(b.size)
        x = X @ xb
        e0 = x @ K @ x
        assert abs(xb @ S @ xb - e0) <= 1e-10 * e0
        for _ in range(3):
            y = x.copy()
            y[i] += 1e-3 * rng.standard_normal(i.size) * np.abs(x).max()
            assert y @ K @ y > e0
        if method == "tfeti":
            Rb = op.R[s][b]
            assert np.abs(S @ Rb).max() <= 1e-10 * np.abs(S).max() * np.abs(Rb).max(), s


def test_superlumped_preconditioner_closed_form_and_convergence(c1):
    """Super-lumped preconditioner (Sec. 3.1: S~^s = diag K_bb). On a homogeneous unit-modulus
    grid, a multiplier row on an interface edge (not a cross point) glues two subdomains whose
    copies of the DOF each sit in two elements, so each K^s_jj = 2 K0_11 and, with weights 1/2,
    (M e_row)_row = 2 (1/2)^2 2 K0_11 = K0_11 = (3 - nu) / (6 (1 - nu^2)) for an x-DOF. With
    heterogeneous densities every variant still reaches the direct solution."""
    prob = workloads.cantilever_tfeti(0, nsub=(2, 1), m=4)
    prob.rho = np.ones_like(prob.rho)
    op = feti.FETIDP(prob, "superlumped", "mult")
    nu = prob.nu
    k11 = (3 - nu) / (6 * (1 - nu ** 2))
    rows = [r for r in range(op.n_lambda) if sum(1 for s in range(len(op.K)) if op.cons.Bb[s][r].nnz) == 2]
    assert rows
    for r in rows:
        e = np.zeros(op.n_lambda)
        e[r] = 1.0
        z = op.precondition(e, one_column=True)[:, 0]
        # x- and y-DOFs of an edge node: K0_11 and K0_22 are equal for the unit square
        assert z[r] == pytest.approx(k11, rel=1e-12)
        # diagonal blocks: no coupling to the neighbouring nodes' rows (the lumped K_bb has it)
        assert np.count_nonzero(z) == 1
    lumped = feti.FETIDP(prob, "lumped", "mult")
    e = np.zeros(op.n_lambda)
    e[rows[0]] = 1.0
    assert np.count_nonzero(lumped.precondition(e, one_column=True)[:, 0]) > 1
    prob, ustar = c1
    for method in ["fetidp", "tfeti"]:
        op = (feti.FETIDP if method == "fetidp" else feti.TFETI)(prob, "superlumped", "k")
        for kr in ["pcg", "sfeti"]:
            res = krylov.solve(op, kr, tol=1e-12)
            assert res.converged
            assert _rel(op.recover(res.lam)[0], ustar) < 1e-8
