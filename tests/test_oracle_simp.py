"""Pins of the oracle's SIMP design update (optimality criteria for minimum compliance under a
volume bound, the application of Sec. 1), no GPU: the volume bound holds after the step, the
move limits and the box [rho_min, 1] hold element by element, the closed form of the multiplier
for a uniform sensitivity without active bounds, and the multiplier against a brute-force scan
of the (monotone) volume function on a small input."""
import numpy as np

from oracle import simp


def test_volume_bound_and_move_limits():
    rng = np.random.default_rng(0)
    rho = rng.uniform(0.0, 1.0, 5000)
    dc = -rng.gamma(0.5, 2.0, 5000) * rho ** 2
    new, lam = simp.oc_update(rho, dc, 0.4, move=0.2, eta=0.5, rho_min=1e-3)
    assert abs(new.sum() - 0.4 * rho.size) <= 1e-9 * rho.size
    assert np.all(new >= np.maximum(1e-3, rho - 0.2) - 1e-15)
    assert np.all(new <= np.minimum(1.0, rho + 0.2) + 1e-15)
    # elements strictly inside their bounds take the unconstrained value rho (|dc| / L)^eta
    lo, hi = np.maximum(1e-3, rho - 0.2), np.minimum(1.0, rho + 0.2)
    inner = (new > lo + 1e-12) & (new < hi - 1e-12)
    assert inner.sum() > 100
    assert np.allclose(new[inner], rho[inner] * np.sqrt(-dc[inner] / lam), rtol=1e-12)


def test_uniform_sensitivity_closed_form():
    # no active bound: rho_new = rho (a / L)^eta, so sum rho_new = V n gives
    # L = a (sum rho / (V n))^(1 / eta)
    rho = np.linspace(0.3, 0.6, 1000)
    a, V, eta = 2.5, 0.46, 0.5
    new, lam = simp.oc_update(rho, -a * np.ones_like(rho), V, move=1.0, eta=eta, rho_min=1e-3)
    lam_exact = a * (rho.sum() / (V * rho.size)) ** (1.0 / eta)
    assert abs(lam - lam_exact) <= 1e-12 * lam_exact
    assert np.allclose(new, rho * (a / lam_exact) ** eta, rtol=1e-12)


def test_multiplier_against_brute_force_scan():
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.05, 0.95, 60)
    dc = -rng.uniform(0.0, 3.0, 60)
    new, lam = simp.oc_update(rho, dc, 0.5, move=0.15, eta=0.5, rho_min=1e-3)
    grid = np.geomspace(1e-6, 1e3, 200001)
    vols = np.array([simp.oc_rho(rho, dc, L, 0.15, 0.5, 1e-3).sum() for L in grid[::100]])
    # volume is non-increasing in L
    assert np.all(np.diff(vols) <= 1e-12)
    target = 0.5 * rho.size
    i = int(np.argmax(vols <= target))
    assert grid[100 * (i - 1)] <= lam <= grid[100 * i]
    assert abs(new.sum() - target) <= 1e-9 * rho.size
