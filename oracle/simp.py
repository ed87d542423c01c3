"""SIMP design update of the oracle (test infrastructure only).

The paper's application (Sec. 1) minimises the compliance c(rho) = f^T u(rho) of the SIMP
system (Eq. 1-2) under a bound on the material volume. It does not state the optimiser; the
reading here is the textbook optimality-criteria (OC) update for that problem with unit
element volumes:

    B_e(L)   = max(0, -dc/drho_e) / L
    rho_e(L) = min(min(1, rho_e + move), max(max(rho_min, rho_e - move), rho_e * B_e(L)^eta))

with the Lagrange multiplier L > 0 of the volume bound chosen so that sum_e rho_e(L) equals
volfrac * n_el. The volume is non-increasing in L; L is bracketed by lo = 0 (every element at
its upper bound) and hi = max_e |dc_e|, doubled until the volume at hi is at most the target,
then bisected: mid = (lo + hi) / 2 replaces hi when the volume at mid is at most the target and
lo otherwise, until hi - lo <= 1e-14 hi or 200 steps. The update uses rho_e(hi).
"""
from __future__ import annotations

import numpy as np


def oc_rho(rho, dc, lam, move, eta, rho_min):
    b = np.maximum(0.0, -dc) / lam
    cand = rho * b ** eta
    lo = np.maximum(rho_min, rho - move)
    hi = np.minimum(1.0, rho + move)
    return np.minimum(hi, np.maximum(lo, cand))


def oc_update(rho, dc, volfrac, move=0.2, eta=0.5, rho_min=1e-3):
    """One OC step; returns (rho_new, L)."""
    rho = np.asarray(rho, dtype=np.float64)
    dc = np.asarray(dc, dtype=np.float64)
    target = volfrac * rho.size
    vol = lambda lam: float(np.sum(oc_rho(rho, dc, lam, move, eta, rho_min)))  # noqa: E731
    lo = 0.0
    hi = float(np.max(np.abs(dc)))
    if not hi > 0.0:
        hi = 1.0
    for _ in range(200):
        if vol(hi) <= target:
            break
        hi *= 2.0
    for _ in range(200):
        if hi - lo <= 1e-14 * hi:
            break
        mid = 0.5 * (lo + hi)
        if vol(mid) <= target:
            hi = mid
        else:
            lo = mid
    return oc_rho(rho, dc, hi, move, eta, rho_min), hi
