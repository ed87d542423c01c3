"""Writes the oracle's runs of the three academic problems of Sec. 4.1 (workloads.ACADEMIC: the
laminated beam, the grid of layered subdomains and the grid of subdomains with stiff inclusions)
for all twelve variants of the paper's comparison: {Total FETI, FETI-DP} x {multiplicity,
k-scaling} x {PCG, full orthogonalisation, simultaneous directions} (Sec. 2-3, Algorithm 1), with
the Dirichlet preconditioner at the relative tolerance 1e-6 (Eq. 16).

Calls only the oracle (``oracle.feti``, ``oracle.krylov``) on the inputs of ``workloads``. For
every run it stores the iteration count, the converged flag and eps_r per iterate; and the same
run on the oracle's operator evaluated through its explicit dense F (the same operator in another
rounding order), whose count measures how far round-off alone moves the oracle's own count; and
the relative distance of the recovered u from the global direct solution.

Usage: python tests/golden/make_academic_goldens.py   (about two minutes on 8 cores)
"""
import pathlib
import sys

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import workloads  # noqa: E402
from oracle import fem, feti, krylov  # noqa: E402

HERE = pathlib.Path(__file__).resolve().parent
TOL = 1e-6


class DenseF:
    """An oracle operator evaluated through its explicit dense F (symmetrised)."""

    def __init__(self, op):
        self.op = op
        F = op.apply_F(np.eye(op.n_lambda))
        self.F = 0.5 * (F + F.T)
        self.n_lambda = op.n_lambda
        self.d = op.d
        self.group = getattr(op, "group", None)
        self.n_groups = getattr(op, "n_groups", None)

    def apply_F(self, L):
        return self.F @ L

    def project(self, Y):
        return self.op.project(Y)

    def lambda0(self):
        return self.op.lambda0()

    def precondition(self, r, one_column=False):
        return self.op.precondition(r, one_column)


def main():
    out = {"tol": TOL}
    for name, gen in workloads.ACADEMIC.items():
        prob = gen()
        u_star = fem.solve_problem(prob)
        for method in ["tfeti", "fetidp"]:
            for scaling in ["mult", "k"]:
                op = (feti.TFETI if method == "tfeti" else feti.FETIDP)(prob, "dirichlet", scaling)
                dop = DenseF(op)
                out[f"{name}_{method}_n_lambda"] = op.n_lambda
                for kr in ["pcg", "fo", "sfeti"]:
                    res = krylov.solve(op, kr, tol=TOL)
                    rd = krylov.solve(dop, kr, tol=TOL)
                    u, _ = op.recover(res.lam)
                    key = f"{name}_{method}_{scaling}_{kr}"
                    out[key + "_iters"] = res.iters
                    out[key + "_converged"] = res.converged
                    out[key + "_history"] = np.asarray(res.history)
                    out[key + "_iters_dense"] = rd.iters
                    out[key + "_u_err"] = np.linalg.norm(u - u_star) / np.linalg.norm(u_star)
                    print(f"{key}: {res.iters} iterations (dense F {rd.iters}), converged {res.converged}",
                          flush=True)
    np.savez(HERE / "academic.npz", **out)


if __name__ == "__main__":
    main()
