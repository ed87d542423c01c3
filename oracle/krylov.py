"""Krylov iterations of the oracle (test infrastructure only).

* ``pcg``: the projected preconditioned conjugate gradient method on the dual
  problem (Sec. 2.1 for TFETI, Sec. 2.2 with u_c condensed out for FETI-DP).
* ``simultaneous``: the rank-revealing simultaneous FETI iteration of Sec. 3.3,
  Algorithm 1. With one direction group it is the fully orthogonalised PCG of
  Sec. 3.2 (the single direction is F-orthonormalised and orthogonalised
  against all stored directions).

The stopping rule: the paper's residual measure is eps_r = sqrt(r_i^T z_i)
(Eq. 16) with z_i = Z_i 1; the threshold is taken relative to its initial value,
eps_r <= tol * eps_0 (the paper gives no value for its threshold epsilon).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Result:
    lam: np.ndarray
    iters: int
    history: list            # eps_r per iterate, starting with eps_0
    converged: bool
    ranks: list = field(default_factory=list)
    status: str = "ok"


def pcg(op, tol=1e-8, max_it=None, Y=None):
    """Projected PCG: r = P(d - F lam), z = M r, w = P z (+ beta w_prev),
    q = F w, a = r^T z / w^T q, lam += a w, r -= a P q. Y (optional): a deflation space
    (oracle.deflation): the start is corrected (deflate) and the new part P z of every direction is
    made F-orthogonal to it (deflated CG); eps_0 is that of the uncorrected start."""
    n = op.n_lambda
    max_it = n if max_it is None else max_it
    lam0 = op.lambda0()
    r = op.project((op.d - op.apply_F(lam0[:, None])[:, 0])[:, None])[:, 0]
    z = op.precondition(r, one_column=True)[:, 0]
    rz = float(r @ z)
    eps0 = np.sqrt(max(rz, 0.0))
    hist = [eps0]
    lt = np.zeros(n)
    Wd, Qd = [], []
    if Y is not None and Y.shape[1] > 0 and eps0 > 0.0:
        Wd, Qd, lt, r = deflate(op, Y, r)
        z = op.precondition(r, one_column=True)[:, 0]
        rz = float(r @ z)

    def deflated(v):
        for Wj, Qj in zip(Wd, Qd):
            v = v - Wj @ (Qj.T @ v)
        return v

    w = deflated(op.project(z[:, None])[:, 0])
    it = 0
    conv = eps0 == 0.0 or np.sqrt(max(rz, 0.0)) <= tol * eps0
    while not conv and it < max_it:
        q = op.apply_F(w[:, None])[:, 0]
        wq = float(w @ q)
        if wq <= 0.0:
            return Result(lam0 + lt, it, hist, False, status="breakdown")
        a = rz / wq
        lt += a * w
        r -= a * op.project(q[:, None])[:, 0]
        z = op.precondition(r, one_column=True)[:, 0]
        rz_new = float(r @ z)
        it += 1
        hist.append(np.sqrt(max(rz_new, 0.0)))
        if hist[-1] <= tol * eps0:
            conv = True
            break
        beta = rz_new / rz
        rz = rz_new
        w = deflated(op.project(z[:, None])[:, 0]) + beta * w
    return Result(lam0 + lt, it, hist, conv)


def pivoted_cholesky(D, rr_tol=1e-12, drop=1e-30):
    """Rank-revealing Cholesky N Dhat N^T = L L^T of the Jacobi-scaled Gram matrix
    Dhat = S^{-1/2} D S^{-1/2}, S = diag D (Sec. 3.3; the paper names the
    factorisation, not its thresholds).

    Columns with D_jj <= drop * max_j D_jj are excluded up front. The pivot is the
    largest remaining diagonal of the Schur complement (lowest column index on
    ties); the factorisation stops when that pivot is <= rr_tol.

    Returns (T, rank) with T = S^{-1/2} N^T [Ltilde^{-T}; 0] of shape [k, rank]:
    W T is the F-orthonormal basis of the kept directions.
    """
    D = np.asarray(D, dtype=np.float64)
    k = D.shape[0]
    dg = np.diag(D).copy()
    dmax = dg.max() if k else 0.0
    if not (dmax > 0.0):
        return np.zeros((k, 0)), 0
    live = [j for j in range(k) if dg[j] > drop * dmax]
    s = np.zeros(k)
    s[live] = 1.0 / np.sqrt(dg[live])
    A = D * s[:, None] * s[None, :]
    order = []
    Lcols = []
    remaining = list(live)
    for _ in range(len(live)):
        # Schur-complement diagonal of the remaining columns
        best, bval = None, -np.inf
        for j in remaining:
            v = A[j, j] - sum(l[j] ** 2 for l in Lcols)
            if v > bval:
                best, bval = j, v
        if bval <= rr_tol:
            break
        piv = np.sqrt(bval)
        l = np.zeros(k)
        l[best] = piv
        for j in remaining:
            if j != best:
                l[j] = (A[j, best] - sum(c[j] * c[best] for c in Lcols)) / piv
        Lcols.append(l)
        order.append(best)
        remaining.remove(best)
    rank = len(order)
    if rank == 0:
        return np.zeros((k, 0)), 0
    Lt = np.array([[Lcols[c][order[r]] for c in range(rank)] for r in range(rank)])
    Linv_T = np.linalg.inv(Lt).T          # rank x rank, upper triangular
    T = np.zeros((k, rank))
    for r in range(rank):
        T[order[r], :] = s[order[r]] * Linv_T[r, :]
    return T, rank


def deflate(op, Y, r, rr_tol=1e-12):
    """F-orthonormal basis of span(P Y) in blocks of 64 columns (each block orthogonalised against
    the previous ones, then F-orthonormalised by the rank-revealing Cholesky of Sec. 3.3) and the
    correction of the start: returns (Wd, Qd, lt, r) with lt = sum_b W_b W_b^T r0 and
    r = r0 - P sum_b Q_b W_b^T r0, so that W_b^T r = 0 for every block."""
    Wd, Qd = [], []
    lt = np.zeros(op.n_lambda)
    for c0 in range(0, Y.shape[1], 64):
        W = op.project(Y[:, c0:c0 + 64])
        for Wj, Qj in zip(Wd, Qd):
            W = W - Wj @ (Qj.T @ W)
        Q = op.apply_F(W)
        D = Q.T @ W
        T, rank = pivoted_cholesky(0.5 * (D + D.T), rr_tol)
        if rank == 0:
            continue
        Wd.append(W @ T)
        Qd.append(Q @ T)
    for Wb, Qb in zip(Wd, Qd):
        g = Wb.T @ r
        lt += Wb @ g
        r = r - op.project(Qb @ g[:, None])[:, 0]
    return Wd, Qd, lt, r


def simultaneous(op, tol=1e-8, max_it=None, rr_tol=1e-12, one_group=False, Y=None):
    """Algorithm 1 (Sec. 3.3). With one_group=True all subdomains feed a single
    column: the fully orthogonalised PCG of Sec. 3.2. Y (n_lambda x m, optional): a deflation
    space (oracle.deflation); its F-orthonormal basis is stored ahead of the iteration's own
    directions and the start is corrected (deflate). eps_0 is that of the uncorrected start, so a
    deflated and a plain solve stop at the same residual measure."""
    n = op.n_lambda
    lam0 = op.lambda0()
    r = op.project((op.d - op.apply_F(lam0[:, None])[:, 0])[:, None])[:, 0]
    Z = op.precondition(r, one_column=one_group)
    eps0 = np.sqrt(max(float(r @ Z.sum(axis=1)), 0.0))
    lt = np.zeros(n)
    Wh, Qh = [], []
    if Y is not None and Y.shape[1] > 0 and eps0 > 0.0:
        Wh, Qh, lt, r = deflate(op, Y, r, rr_tol)
        Z = op.precondition(r, one_column=one_group)
    W = op.project(Z)
    for Wj, Qj in zip(Wh, Qh):
        W = W - Wj @ (Qj.T @ W)
    hist = [eps0]
    ranks = []
    it = 0
    kept = sum(Wj.shape[1] for Wj in Wh)
    max_it = n if max_it is None else max_it
    status = "ok"
    conv = eps0 == 0.0 or np.sqrt(max(float(r @ Z.sum(axis=1)), 0.0)) <= tol * eps0
    while not conv and it < max_it and kept < n:
        Q = op.apply_F(W)
        Delta = Q.T @ W
        T, rank = pivoted_cholesky(0.5 * (Delta + Delta.T), rr_tol)
        ranks.append(rank)
        if rank == 0:
            status = "breakdown"
            break
        W = W @ T
        Q = Q @ T
        gamma = W.T @ r
        lt += W @ gamma
        r = r - op.project(Q @ gamma[:, None])[:, 0]
        Wh.append(W)
        Qh.append(Q)
        kept += rank
        Z = op.precondition(r, one_column=one_group)
        W = op.project(Z)
        for Wj, Qj in zip(Wh, Qh):
            Psi = Qj.T @ W
            W = W - Wj @ Psi
        it += 1
        hist.append(np.sqrt(max(float(r @ Z.sum(axis=1)), 0.0)))
        if hist[-1] <= tol * eps0:
            conv = True
    return Result(lam0 + lt, it, hist, conv, ranks, status)


def solve(op, krylov="pcg", tol=1e-8, max_it=None, rr_tol=1e-12, Y=None):
    if krylov == "pcg":
        return pcg(op, tol, max_it, Y=Y)
    if krylov == "fo":
        return simultaneous(op, tol, max_it, rr_tol, one_group=True, Y=Y)
    if krylov == "sfeti":
        return simultaneous(op, tol, max_it, rr_tol, one_group=False, Y=Y)
    raise ValueError(krylov)
