"""Deflation of local interface modes (test infrastructure only).

The paper names this only as further work (Sec. 6, item (ii)): find the interface modes
responsible for slow convergence and remove them from the iterative process, in the manner of
GenEO. It fixes neither the local problem nor the selection; the reading taken here:

* Local problem. For subdomain s, with R_s the dual rows it touches, B_s its signed boolean map
  from its interface DOFs to those rows and w_s its weights on them (the scaling of the
  preconditioner), the subdomain contributes
      P_s = diag(w_s) B_s S_s B_s^T diag(w_s)      to the preconditioner (S_s the preconditioner
                                                    block: Dirichlet Schur complement, K_bb, or
                                                    its diagonal), and
      F_s = B_s Fl_s B_s^T                          to the dual operator (Fl_s: TFETI B K^+ B^T
                                                    block, FETI-DP the K_rr^{-1} interface block).
  Its bad modes are the eigenvectors of the local preconditioned operator P_s F_s with the largest
  eigenvalues mu: directions on which the preconditioner over-weights the subdomain's stiffness.
  With Fl_s = L L^T (any square-root factor) and G = B_s L, the nonzero eigenvalues of
  P_s F_s = P_s G G^T are those of the symmetric C_s = G^T P_s G = L^T (omega S_s omega) L (omega = B_s^T diag(w_s) B_s, diagonal:
  the summed weights of each interface DOF), and for C_s x = mu x the vector y = P_s G x is an
  eigenvector of P_s F_s: y = diag(w_s) B_s u with u = S_s omega L x.
* Selection: an invariant subspace of at most m modes per subdomain that is unique: the k largest
  mu, k the largest count <= m whose k-th eigenvalue lies above both the threshold tau and a
  relative gap, mu_k >= (1 + gap) mu_{k+1} (mu_{k+1} = 0 past the spectrum). A cluster of equal
  eigenvalues is taken whole or not at all, so any eigensolver selects the same space.
* Deflation: the span of the y of all subdomains is made F-orthonormal (in blocks of 64 columns,
  each orthogonalised against the previous blocks and F-orthonormalised by the rank-revealing
  Cholesky of Sec. 3.3), the start is corrected so that the residual is orthogonal to it, and the
  Krylov iteration orthogonalises its directions against it as against its own stored ones
  (krylov.simultaneous with Y).
"""
from __future__ import annotations

import numpy as np


def select_count(mu_desc, m, tau=0.0, gap=0.05):
    """Number k of leading modes taken from eigenvalues sorted in decreasing order: the largest
    k <= m with mu_k >= tau and mu_k >= (1 + gap) mu_{k+1}, or 0."""
    for k in range(min(m, len(mu_desc)), 0, -1):
        nxt = mu_desc[k] if k < len(mu_desc) else 0.0
        if mu_desc[k - 1] >= tau and mu_desc[k - 1] >= (1.0 + gap) * nxt:
            return k
    return 0


def local_modes(op, s, m, tau=0.0, gap=0.05):
    """(mu, U, Y) of subdomain s: the selected largest eigenvalues mu of its local preconditioned
    operator (select_count), the interface-DOF vectors u = S_s omega L x and the dual vectors
    y = diag(w_s) B_s u (length n_lambda, zero off the rows of s)."""
    Bb = op.cons.Bb[s]
    rows = np.unique(Bb.nonzero()[0])
    if rows.size == 0 or m <= 0:
        return np.zeros(0), np.zeros((Bb.shape[1], 0)), np.zeros((op.n_lambda, 0))
    Bs = Bb[rows].toarray()
    w = op.w[s][rows]
    # a square-root factor Fl = L L^T from the eigendecomposition, so that a semi-definite Fl
    # (TFETI: the pseudo-inverse of a floating subdomain) is covered too; any other factor
    # L Q (Q orthogonal) gives the same mu and u
    lam, V = np.linalg.eigh(0.5 * (op.F_local[s] + op.F_local[s].T))
    keep = lam > 1e-13 * max(lam.max(), 0.0)
    L = V[:, keep] * np.sqrt(lam[keep])[None, :]
    omega = np.diag(Bs.T @ (w[:, None] * Bs))
    S = np.asarray(op.S[s])
    C = L.T @ (omega[:, None] * S * omega[None, :]) @ L
    mu, X = np.linalg.eigh(0.5 * (C + C.T))
    desc = np.argsort(mu)[::-1]
    order = desc[:select_count(mu[desc], m, tau, gap)]
    U = S @ (omega[:, None] * (L @ X[:, order]))
    Y = np.zeros((op.n_lambda, order.size))
    Y[rows] = w[:, None] * (Bs @ U)
    return mu[order], U, Y


def deflation_space(op, m, tau=0.0, gap=0.05):
    """Y = [y of subdomain 0 | y of subdomain 1 | ...] and the eigenvalues, subdomain by subdomain."""
    mus, Ys = [], []
    for s in range(len(op.dec.subs)):
        mu, _, Y = local_modes(op, s, m, tau, gap)
        mus.append(mu)
        Ys.append(Y)
    return np.hstack(Ys) if Ys else np.zeros((op.n_lambda, 0)), mus
