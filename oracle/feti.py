"""Dual operators of the oracle (test infrastructure only).

Total FETI (Sec. 2.1): F = B K^+ B^T, d = B K^+ f - c, G = -R^T B^T, e = -R^T f
(Eq. 7) with K^+ the exact Moore-Penrose pseudo-inverse of every floating
subdomain, K^+ = (K + tau R R^T)^{-1} - R R^T / tau for orthonormal R.

FETI-DP (Sec. 2.2): F_rr = B_r K_rr^{-1} B_r^T, F_rc = B_r K_rr^{-1} K_rc,
Kbar_cc = K_cc - K_cr K_rr^{-1} K_rc, d_r = B_r K_rr^{-1} f_r,
fbar_c = f_c - K_cr K_rr^{-1} f_r (Eq. 12). Eliminating u_c from the second row
of Eq. (12), u_c = Kbar_cc^{-1} (fbar_c + F_rc^T lambda), leaves the lambda-only
system (F_rr + F_rc Kbar_cc^{-1} F_rc^T) lambda = d_r - F_rc Kbar_cc^{-1} fbar_c.

Preconditioner (Sec. 3.1, Eq. 13): sum_s B~^s S~^s B~^sT with B~^s = W^s B^s and
S~^s the Dirichlet Schur complement K_bb - K_bi K_ii^{-1} K_ib, the lumped K_bb or the
super-lumped diag K_bb;
in FETI-DP the sets i and b are subsets of r. For simultaneous directions the
contribution of subdomain s goes to column g(s) of Z (Algorithm 1).

Everything is built from sparse per-subdomain stiffness matrices with scipy's
sparse LU; the explicit local matrices F_s are dense numpy arrays.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads

from . import fem, topology


def subdomain_stiffness(prob, sd, E, K0):
    """K^s = sum over the subdomain's elements of E_e K0 (Sec. 2, Eq. 3)."""
    ed = sd.elem_ldofs
    n = sd.n_loc
    rows = np.repeat(ed, ed.shape[1], axis=1).ravel()
    cols = np.tile(ed, (1, ed.shape[1])).ravel()
    vals = (E[sd.elems][:, None] * K0.ravel()[None, :]).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def split_load(dec, f):
    """Local loads f^s: a global load entry goes wholly to the lowest-numbered
    subdomain containing its node (any split gives the same u)."""
    n_sub = len(dec.subs)
    owner = {}
    for sd in dec.subs:
        for l, g in enumerate(sd.dofs):
            owner.setdefault(int(g), (sd.index, l))
    fs = [np.zeros(sd.n_loc) for sd in dec.subs]
    for g in np.nonzero(f)[0]:
        s, l = owner[int(g)]
        fs[s][l] += f[g]
    return fs


def schur_on(Ks, b_idx, active_idx):
    """Dirichlet Schur complement onto b of K restricted to the active index set."""
    i_idx = np.setdiff1d(active_idx, b_idx)
    Kbb = Ks[b_idx][:, b_idx].toarray()
    if i_idx.size == 0:
        return Kbb
    Kii = Ks[i_idx][:, i_idx].tocsc()
    Kib = Ks[i_idx][:, b_idx].toarray()
    X = spla.splu(Kii).solve(Kib)
    return Kbb - Kib.T @ X


def fetidp_local(Ks, r, c, bpos):
    """Local FETI-DP operators of one subdomain (Sec. 2.2, Eq. 11-12): with Y = K_rr^{-1} [E_b, K_rc]
    (E_b the unit columns of the interface positions bpos within r), F_s = (K_rr^{-1})_bb,
    F_rc^s = (K_rr^{-1} K_rc)_b and Kbar_cc^s = K_cc - K_cr K_rr^{-1} K_rc. Returns
    (F_s, F_rc^s, Kbar_cc^s, K_rc, LU of K_rr)."""
    Krr = Ks[r][:, r].tocsc()
    Krc = Ks[r][:, c].toarray()
    Kcc = Ks[c][:, c].toarray()
    lu = _LU(Krr)
    Eb = np.zeros((r.size, bpos.size))
    Eb[bpos, np.arange(bpos.size)] = 1.0
    Y = lu.solve(np.hstack([Eb, Krc]))
    Yc = Y[:, bpos.size:]
    return Y[bpos, :bpos.size], Yc[bpos], Kcc - Krc.T @ Yc, Krc, lu


class _Common:
    """Weights, preconditioner and direction groups shared by both methods."""

    def _setup_precond(self, precond, scaling, active_sets):
        self.precond_kind = precond
        self.scaling_kind = scaling
        self.S = []
        for s, sd in enumerate(self.dec.subs):
            b_loc = self.b_local[s]
            if precond == "dirichlet":
                self.S.append(schur_on(self.K[s], b_loc, active_sets[s]))
            elif precond == "lumped":
                self.S.append(self.K[s][b_loc][:, b_loc].toarray())
            elif precond == "superlumped":
                self.S.append(np.diag(self.K[s][b_loc][:, b_loc].diagonal()))
            else:
                raise ValueError(precond)
        col_to_local = self.col_to_local

        def diag_of(s, col):
            l = col_to_local[s][col]
            return self.K[s][l, l]

        self.w = topology.scaling_weights(self.cons, diag_of, scaling)
        self.group = workloads.group_of_subdomains(self.prob.nsub, self.prob.groups)
        self.n_groups = int(self.group.max()) + 1

    @property
    def n_lambda(self):
        return self.cons.n_rows

    def precondition(self, r, one_column=False):
        """Z = [.., B~^s S~^s B~^sT r, ..] summed per direction group (Algorithm 1);
        with one_column the plain preconditioned residual z = Z 1 (Eq. 13)."""
        k = 1 if one_column else self.n_groups
        Z = np.zeros((self.n_lambda, k))
        for s in range(len(self.dec.subs)):
            Bb = self.cons.Bb[s]
            x = Bb.T @ (self.w[s] * r)
            y = self.S[s] @ x
            col = 0 if one_column else self.group[s]
            Z[:, col] += self.w[s] * (Bb @ y)
        return Z


class TFETI(_Common):
    """Total FETI operators (Sec. 2.1)."""

    def __init__(self, prob, precond="lumped", scaling="mult"):
        self.prob = prob
        self.dec = topology.decompose(prob)
        self.cons = topology.tfeti_constraints(self.dec)
        E = fem.simp_modulus(prob.rho, prob.p, prob.E0, prob.Emin)
        K0 = fem.element_stiffness(prob.dim, prob.nu)
        self.K = [subdomain_stiffness(prob, sd, E, K0) for sd in self.dec.subs]
        self.f = prob.load()
        self.fs = split_load(self.dec, self.f)
        self.R = [topology.rigid_body_modes(prob, sd) for sd in self.dec.subs]
        self.Kdag = []
        for Ks, R in zip(self.K, self.R):
            A = Ks.toarray()
            tau = float(np.mean(np.diag(A)))
            self.Kdag.append(np.linalg.inv(A + tau * R @ R.T) - R @ R.T / tau)
        self.b_local = self.cons.bset
        self.col_to_local = [np.arange(sd.n_loc) for sd in self.dec.subs]
        self.F_local = [Kd[b][:, b] for Kd, b in zip(self.Kdag, self.b_local)]
        self._setup_precond(precond, scaling, [np.arange(sd.n_loc) for sd in self.dec.subs])
        # G = -R^T B^T, e = -R^T f
        self.G = np.vstack([-(self.cons.B[s] @ self.R[s]).T for s in range(len(self.K))])
        self.e = np.concatenate([-(self.R[s].T @ self.fs[s]) for s in range(len(self.K))])
        self.GGt = self.G @ self.G.T
        self.GGt_cho = sla.cho_factor(self.GGt)
        self.d = sum(self.cons.B[s] @ (self.Kdag[s] @ self.fs[s]) for s in range(len(self.K)))

    def apply_F(self, L):
        """F Lambda = sum_s B^s K^s+ B^sT Lambda, via the b-blocks F_s = (K^s+)_bb."""
        L = np.asarray(L, dtype=np.float64)
        Q = np.zeros_like(L)
        for s in range(len(self.K)):
            Bb = self.cons.Bb[s]
            Q += Bb @ (self.F_local[s] @ (Bb.T @ L))
        return Q

    def project(self, Y):
        """P Y = Y - G^T (G G^T)^{-1} G Y (Sec. 3.3)."""
        return Y - self.G.T @ sla.cho_solve(self.GGt_cho, self.G @ Y)

    def lambda0(self):
        """Minimum-norm lambda with G lambda = e."""
        return self.G.T @ sla.cho_solve(self.GGt_cho, self.e)

    def recover(self, lam):
        """alpha = (G G^T)^{-1} G (d - F lambda); u^s = K^s+ (f^s - B^sT lambda) + R^s alpha^s;
        global u = average of the subdomain copies."""
        res = self.d - self.apply_F(lam[:, None])[:, 0]
        alpha = sla.cho_solve(self.GGt_cho, self.G @ res)
        nm = self.R[0].shape[1]
        us = []
        for s in range(len(self.K)):
            us.append(self.Kdag[s] @ (self.fs[s] - self.cons.B[s].T @ lam) + self.R[s] @ alpha[nm * s:nm * (s + 1)])
        return average_copies(self.dec, us), us


class FETIDP(_Common):
    """FETI-DP operators (Sec. 2.2) with u_c condensed out."""

    def __init__(self, prob, precond="dirichlet", scaling="mult", primal_nodes=None):
        self.prob = prob
        self.dec = topology.decompose(prob, primal_nodes)
        self.split, self.cons = topology.fetidp_split(self.dec)
        E = fem.simp_modulus(prob.rho, prob.p, prob.E0, prob.Emin)
        K0 = fem.element_stiffness(prob.dim, prob.nu)
        self.K = [subdomain_stiffness(prob, sd, E, K0) for sd in self.dec.subs]
        self.f = prob.load()
        self.fs = split_load(self.dec, self.f)
        n_sub = len(self.K)
        self.lu, self.F_local, self.Frc, self.Kcc_bar, self.Krc = [], [], [], [], []
        self.b_local = []
        self.col_to_local = []
        fbar_c = np.zeros(self.split.corner_dofs.size)
        d_r = np.zeros(self.cons.n_rows)
        for s in range(n_sub):
            r, c = self.split.r[s], self.split.c[s]
            bpos = self.cons.bset[s]                 # positions in r
            Fs, Frc, Kcc_bar, Krc, lu = fetidp_local(self.K[s], r, c, bpos)
            self.F_local.append(Fs)
            self.Frc.append(Frc)
            self.Kcc_bar.append(Kcc_bar)
            self.Krc.append(Krc)
            self.lu.append(lu)
            self.b_local.append(r[bpos])
            self.col_to_local.append(r)
            fr = self.fs[s][r]
            xr = lu.solve(fr)
            d_r += self.cons.B[s] @ xr
            fbar_c += self.split.Bc[s].T @ (self.fs[s][c] - Krc.T @ xr)
        self.n_cg = self.split.corner_dofs.size
        # Kbar_cc = sum_s B_c^sT Kbar_cc^s B_c^s (Eq. 11 definitions, then Eq. 12)
        self.Kcc_glob = np.zeros((self.n_cg, self.n_cg))
        for s in range(n_sub):
            Bc = self.split.Bc[s].toarray()
            self.Kcc_glob += Bc.T @ self.Kcc_bar[s] @ Bc
        self.Kcc_cho = sla.cho_factor(self.Kcc_glob) if self.n_cg else None
        self.fbar_c = fbar_c
        self.d_r = d_r
        self._setup_precond(precond, scaling, [self.split.r[s] for s in range(n_sub)])
        self.d = self.d_r - self.apply_Frc(self.coarse_solve(self.fbar_c[:, None]))[:, 0]

    def coarse_solve(self, t):
        if self.n_cg == 0:
            return np.zeros((0, t.shape[1]))
        return sla.cho_solve(self.Kcc_cho, t)

    def apply_Frr(self, L):
        Q = np.zeros_like(L)
        for s in range(len(self.K)):
            Bb = self.cons.Bb[s]
            Q += Bb @ (self.F_local[s] @ (Bb.T @ L))
        return Q

    def apply_FrcT(self, L):
        """F_rc^T Lambda = sum_s B_c^sT F_rc^sT B_r^sT Lambda  ([n_cg, k])."""
        t = np.zeros((self.n_cg, L.shape[1]))
        for s in range(len(self.K)):
            t += self.split.Bc[s].T @ (self.Frc[s].T @ (self.cons.Bb[s].T @ L))
        return t

    def apply_Frc(self, V):
        Q = np.zeros((self.n_lambda, V.shape[1]))
        for s in range(len(self.K)):
            Q += self.cons.Bb[s] @ (self.Frc[s] @ (self.split.Bc[s] @ V))
        return Q

    def apply_F(self, L):
        """F_DP Lambda = F_rr Lambda + F_rc Kbar_cc^{-1} F_rc^T Lambda."""
        L = np.asarray(L, dtype=np.float64)
        return self.apply_Frr(L) + self.apply_Frc(self.coarse_solve(self.apply_FrcT(L)))

    def project(self, Y):
        return Y

    def lambda0(self):
        return np.zeros(self.n_lambda)

    def recover(self, lam):
        """u_c = Kbar_cc^{-1} (fbar_c + F_rc^T lambda);
        u_r^s = K_rr^{-1} (f_r^s - K_rc^s B_c^s u_c - B_r^sT lambda); clamped DOFs 0."""
        uc = self.coarse_solve((self.fbar_c + self.apply_FrcT(lam[:, None])[:, 0])[:, None])[:, 0]
        us = []
        for s, sd in enumerate(self.dec.subs):
            r, c = self.split.r[s], self.split.c[s]
            ucs = self.split.Bc[s] @ uc
            rhs = self.fs[s][r] - self.Krc[s] @ ucs - self.cons.B[s].T @ lam
            u = np.zeros(sd.n_loc)
            u[r] = self.lu[s].solve(rhs)
            u[c] = ucs
            us.append(u)
        return average_copies(self.dec, us), us


class _LU:
    """Sparse LU of K_rr^s that also accepts an empty remainder set."""

    def __init__(self, A):
        self.n = A.shape[0]
        self.lu = spla.splu(A) if self.n else None

    def solve(self, b):
        b = np.asarray(b, dtype=np.float64)
        if self.n == 0:
            return np.zeros_like(b)
        return self.lu.solve(b)


def average_copies(dec, us):
    n = dec.prob.n_dof
    acc = np.zeros(n)
    cnt = np.zeros(n)
    for sd, u in zip(dec.subs, us):
        np.add.at(acc, sd.dofs, u)
        np.add.at(cnt, sd.dofs, 1.0)
    return acc / np.maximum(cnt, 1.0)
