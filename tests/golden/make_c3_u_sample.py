"""Writes c3_u_sample.npz: the global direct solution u* of the 16x16-subdomain cantilever of
64x64 Q4 elements with rho ~ Beta(0.3, 0.3) and Emin/E0 = 1e-9 (2 101 250 DOFs), at 4096 seeded
sample DOFs, with its full Euclidean norm.

Calls only the oracle: assembly of the global K and a sparse LU of its free block
(about 7 minutes and 20 GB on the host). Run from anywhere: python tests/golden/make_c3_u_sample.py
"""
import pathlib
import sys

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import workloads  # noqa: E402
from oracle import fem  # noqa: E402


def main():
    prob = workloads.beta_2d(0)
    u = fem.solve_problem(prob)
    rng = np.random.default_rng(2111)
    idx = np.sort(rng.choice(prob.n_dof, 4096, replace=False))
    np.savez(pathlib.Path(__file__).with_name("c3_u_sample.npz"), idx=idx, u=u[idx], norm=np.linalg.norm(u),
             n_dof=prob.n_dof)


if __name__ == "__main__":
    main()
