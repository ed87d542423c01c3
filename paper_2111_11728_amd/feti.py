"""Python binding of the C ABI in include/feti.h (argument marshalling only).

Every function here has the name of the C entry point it calls; array arguments are
torch tensors on the GPU (their data_ptr() is passed) and the current torch stream is
used. All arithmetic happens in the HIP library; if libfeti.so is missing the import
fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfeti.so")

# ---- constants (feti.h) ----
FETI_OK, FETI_EINVAL, FETI_ENOMEM, FETI_EHIP, FETI_ENOTSPD, FETI_ENOCONV, FETI_EBREAKDOWN = 0, -1, -2, -3, -4, -5, -6
FETI_TFETI, FETI_DP = 0, 1
FETI_MULT, FETI_KSCALE = 0, 1
FETI_PCG, FETI_FO, FETI_SFETI = 0, 1, 2
FETI_DIRICHLET, FETI_LUMPED, FETI_SUPERLUMPED = 0, 1, 2
FETI_FP64, FETI_FP32, FETI_BF16X3 = 0, 1, 2
FETI_PURE = 16
FETI_PRECOND_FP32 = 2

METHODS = {"tfeti": FETI_TFETI, "fetidp": FETI_DP}
SCALINGS = {"mult": FETI_MULT, "k": FETI_KSCALE}
KRYLOVS = {"pcg": FETI_PCG, "fo": FETI_FO, "sfeti": FETI_SFETI}
PRECONDS = {"dirichlet": FETI_DIRICHLET, "lumped": FETI_LUMPED, "superlumped": FETI_SUPERLUMPED}
PRECISIONS = {"fp64": FETI_FP64, "fp32": FETI_FP32, "bf16x3": FETI_BF16X3}


class feti_mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("nel", C.c_int * 3), ("nu", C.c_double), ("n_fixed", C.c_int),
                ("fixed_dofs", C.POINTER(C.c_int))]


class feti_partition(C.Structure):
    _fields_ = [("nsub", C.c_int * 3), ("cuts", C.POINTER(C.c_int) * 3), ("group", C.c_int * 3),
                ("n_primal", C.c_int), ("primal_nodes", C.POINTER(C.c_int))]


class feti_opts(C.Structure):
    _fields_ = [("method", C.c_int), ("scaling", C.c_int), ("krylov", C.c_int), ("precond", C.c_int),
                ("precision", C.c_int), ("tol", C.c_double), ("max_it", C.c_int), ("rr_tol", C.c_double),
                ("reorth", C.c_int), ("max_refine", C.c_int), ("relax", C.c_double), ("graphs", C.c_int),
                ("orth_fp32", C.c_int), ("warm_start", C.c_int), ("recycle", C.c_int), ("defl_modes", C.c_int),
                ("defl_tau", C.c_double), ("precond_fp32", C.c_int)]


class feti_info(C.Structure):
    _fields_ = [("iters", C.c_int), ("refinements", C.c_int), ("status", C.c_int), ("eps0", C.c_double),
                ("eps", C.c_double), ("true_rel_res", C.c_double), ("kept_directions", C.c_int),
                ("res_hist", C.POINTER(C.c_double)), ("res_hist_cap", C.c_int), ("rank_hist", C.POINTER(C.c_int)),
                ("t_solve_ms", C.c_double), ("fp64_fallback", C.c_int),
                ("reduced_iters", C.c_int), ("precision_probes", C.c_int), ("reduced_rel_err", C.c_double),
                ("reduced_orth_err", C.c_double)]


class feti_design(C.Structure):
    _fields_ = [("el0", C.c_longlong), ("n_el", C.c_longlong), ("dof0", C.c_longlong), ("n_dof", C.c_longlong),
                ("sub0", C.c_int), ("n_sub", C.c_int), ("lam0", C.c_int), ("n_lambda", C.c_int),
                ("n_groups", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class feti_tuning(C.Structure):
    _fields_ = [("max_red", C.c_int), ("max_d", C.c_int), ("xcd", C.c_int), ("split_d", C.c_int),
                ("us", C.c_double), ("us_default", C.c_double), ("from_cache", C.c_int), ("fp64_first", C.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class feti_sizes(C.Structure):
    _fields_ = [("n_sub", C.c_int), ("n_dof", C.c_int), ("n_el", C.c_int), ("n_lambda", C.c_int), ("n_cg", C.c_int),
                ("n_alpha", C.c_int), ("n_groups", C.c_int), ("nb_max", C.c_int), ("nb_min", C.c_int),
                ("n_loc_max", C.c_int), ("n_i_max", C.c_int), ("band_max", C.c_int), ("sum_nb2", C.c_longlong),
                ("sum_nb_nc", C.c_longlong), ("device_bytes", C.c_longlong), ("n_fp64_subs", C.c_int),
                ("n_designs", C.c_int), ("sum_nb2_fp64", C.c_longlong), ("n_setup_subs", C.c_int),
                ("n_defl", C.c_int), ("n_defl_kept", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2111_11728_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I, D, LL = C.c_void_p, C.c_int, C.c_double, C.c_longlong
        sig = {
            "feti_plan_sizes": (I, [C.POINTER(feti_mesh), C.POINTER(feti_partition), C.POINTER(feti_opts),
                                    C.POINTER(feti_sizes)]),
            "feti_plan_export": (I, [C.POINTER(feti_mesh), C.POINTER(feti_partition), C.POINTER(feti_opts), I,
                                     C.POINTER(C.c_int), LL, C.POINTER(LL)]),
            "feti_setup": (I, [C.POINTER(feti_mesh), C.POINTER(feti_partition), C.POINTER(feti_opts), P, D, D, D, P,
                               C.POINTER(P)]),
            "feti_update_rho": (I, [P, P]),
            "feti_solve": (I, [P, P, P, P, C.POINTER(feti_info)]),
            "feti_compliance_and_grad": (I, [P, P, P, P, P, P, C.POINTER(feti_info)]),
            "feti_destroy": (I, [P]),
            "feti_last_error": (C.c_char_p, []),
            "feti_get_sizes": (I, [P, C.POINTER(feti_sizes)]),
            "feti_apply_F": (I, [P, I, I, P, P]),
            "feti_get_lambda": (I, [P, P]),
            "feti_get_deflation": (I, [P, P, P]),
            "feti_oc_update": (I, [P, P, P, D, D, D, D, P, C.POINTER(C.c_double)]),
            "feti_adaptive_primal": (I, [C.POINTER(feti_mesh), C.POINTER(feti_partition), P, D, D, D, D, I,
                                         C.POINTER(C.c_int), I, C.POINTER(C.c_int)]),
            "feti_apply_F_noalloc": (I, [P, I, I, P, P]),
            "feti_apply_precond": (I, [P, P, P, I]),
            "feti_project": (I, [P, I, P]),
            "feti_rhs": (I, [P, P, P, P]),
            "feti_get_local": (I, [P, I, I, C.POINTER(D), LL, C.POINTER(I), C.POINTER(I)]),
            "feti_last_timing": (I, [P, I, C.POINTER(D)]),
            "feti_setup_batched": (I, [I, C.POINTER(feti_mesh), C.POINTER(feti_partition), C.POINTER(feti_opts), P,
                                       D, D, D, P, C.POINTER(P)]),
            "feti_design_layout": (I, [P, I, C.POINTER(feti_design)]),
            "feti_design_residuals": (I, [P, C.POINTER(D), I]),
            "feti_autotune": (I, [P, I, C.c_char_p, C.POINTER(feti_tuning)]),
            "feti_set_tuning": (I, [P, C.POINTER(feti_tuning)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class FetiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"feti status {status}: {msg}")
        self.status = status


def _check(st, allow=()):
    if st != FETI_OK and st not in allow:
        raise FetiError(st, lib().feti_last_error().decode())
    return st


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Spec:
    """ctypes views of a workloads.Problem (keeps the host arrays alive)."""

    def __init__(self, prob, method="fetidp", scaling="k", krylov="pcg", precond="dirichlet", precision="fp64",
                 tol=1e-8, max_it=0, rr_tol=0.0, reorth=0, max_refine=-1, relax=0.0, graphs=0, orth_fp32=0,
                 primal_nodes=None, warm_start=0, recycle=0, defl_modes=0, defl_tau=0.0, precond_fp32=0):
        self.prob = prob
        fixed = np.ascontiguousarray(prob.fixed_dofs(), dtype=np.int32)
        self._fixed = fixed
        self.mesh = feti_mesh()
        self.mesh.dim = prob.dim
        for a in range(3):
            self.mesh.nel[a] = prob.nel[a] if a < prob.dim else 0
        self.mesh.nu = prob.nu
        self.mesh.n_fixed = fixed.size
        self.mesh.fixed_dofs = fixed.ctypes.data_as(C.POINTER(C.c_int))
        self.part = feti_partition()
        self._cuts = []
        for a in range(3):
            if a < prob.dim:
                cu = np.ascontiguousarray(prob.cuts[a], dtype=np.int32)
                self._cuts.append(cu)
                self.part.nsub[a] = cu.size - 1
                self.part.cuts[a] = cu.ctypes.data_as(C.POINTER(C.c_int))
            else:
                self.part.nsub[a] = 1
                self.part.cuts[a] = C.POINTER(C.c_int)()
            self.part.group[a] = (prob.groups[a] if (prob.groups is not None and a < prob.dim) else 0)
        self._primal = np.ascontiguousarray(np.asarray([] if primal_nodes is None else primal_nodes), dtype=np.int32)
        self.part.n_primal = self._primal.size
        self.part.primal_nodes = (self._primal.ctypes.data_as(C.POINTER(C.c_int)) if self._primal.size
                                  else C.POINTER(C.c_int)())
        self.opts = feti_opts(METHODS[method], SCALINGS[scaling], KRYLOVS[krylov], PRECONDS[precond],
                              PRECISIONS[precision], tol, max_it, rr_tol, reorth, max_refine, relax, graphs,
                              orth_fp32, warm_start, recycle, defl_modes, defl_tau, int(precond_fp32))


def feti_plan_sizes(spec: Spec) -> dict:
    out = feti_sizes()
    _check(lib().feti_plan_sizes(C.byref(spec.mesh), C.byref(spec.part), C.byref(spec.opts), C.byref(out)))
    return out.as_dict()


def feti_adaptive_primal(spec: Spec, theta=0.2, cap=3) -> np.ndarray:
    """Host-only: the library's adaptive choice of further FETI-DP primal nodes for spec's
    problem (its densities and SIMP parameters)."""
    prob = spec.prob
    rho = np.ascontiguousarray(prob.rho, dtype=np.float64)
    n = C.c_int(0)
    rp = C.c_void_p(rho.ctypes.data)
    _check(lib().feti_adaptive_primal(C.byref(spec.mesh), C.byref(spec.part), rp, prob.p, prob.E0, prob.Emin,
                                      theta, cap, None, 0, C.byref(n)))
    buf = np.zeros(max(1, n.value), dtype=np.int32)
    _check(lib().feti_adaptive_primal(C.byref(spec.mesh), C.byref(spec.part), rp, prob.p, prob.E0, prob.Emin,
                                      theta, cap, buf.ctypes.data_as(C.POINTER(C.c_int)), buf.size, C.byref(n)))
    return buf[:n.value].astype(np.int64)


def feti_plan_export(spec: Spec, what: int) -> np.ndarray:
    n = C.c_longlong(0)
    _check(lib().feti_plan_export(C.byref(spec.mesh), C.byref(spec.part), C.byref(spec.opts), what, None, 0,
                                  C.byref(n)), allow=(FETI_EINVAL,))
    buf = np.zeros(max(1, n.value), dtype=np.int32)
    _check(lib().feti_plan_export(C.byref(spec.mesh), C.byref(spec.part), C.byref(spec.opts), what,
                                  buf.ctypes.data_as(C.POINTER(C.c_int)), buf.size, C.byref(n)))
    return buf[:n.value]


class Context:
    """Owns one feti_ctx (feti_setup ... feti_destroy)."""

    def __init__(self, spec: Spec, rho, p=None, E0=None, Emin=None):
        prob = spec.prob
        self.spec = spec
        self.p = prob.p if p is None else p
        self.E0 = prob.E0 if E0 is None else E0
        self.Emin = prob.Emin if Emin is None else Emin
        self.handle = C.c_void_p()
        _check(lib().feti_setup(C.byref(spec.mesh), C.byref(spec.part), C.byref(spec.opts), _ptr(rho), self.p,
                                self.E0, self.Emin, _stream(), C.byref(self.handle)))
        self.sizes = self.feti_get_sizes()

    def close(self):
        if self.handle:
            lib().feti_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def feti_get_sizes(self) -> dict:
        out = feti_sizes()
        _check(lib().feti_get_sizes(self.handle, C.byref(out)))
        return out.as_dict()

    def feti_update_rho(self, rho):
        _check(lib().feti_update_rho(self.handle, _ptr(rho)))

    def feti_solve(self, f, u, lambda_init=None, hist_cap=4096, allow_noconv=False):
        info = feti_info()
        hist = np.zeros(hist_cap)
        ranks = np.zeros(hist_cap, dtype=np.int32)
        info.res_hist = hist.ctypes.data_as(C.POINTER(C.c_double))
        info.rank_hist = ranks.ctypes.data_as(C.POINTER(C.c_int))
        info.res_hist_cap = hist_cap
        allow = (FETI_ENOCONV, FETI_EBREAKDOWN) if allow_noconv else ()
        st = _check(lib().feti_solve(self.handle, _ptr(f), _ptr(u), _ptr(lambda_init), C.byref(info)), allow=allow)
        n = min(hist_cap, info.iters + 1)
        return {"status": st, "iters": info.iters, "refinements": info.refinements, "eps0": info.eps0,
                "eps": info.eps, "true_rel_res": info.true_rel_res, "kept_directions": info.kept_directions,
                "history": hist[:n].copy(), "ranks": ranks[:info.iters].copy(), "t_solve_ms": info.t_solve_ms,
                "fp64_fallback": info.fp64_fallback, "reduced_iters": info.reduced_iters,
                "precision_probes": info.precision_probes, "reduced_rel_err": info.reduced_rel_err,
                "reduced_orth_err": info.reduced_orth_err}

    def feti_compliance_and_grad(self, rho, f, c, dc, u=None, allow_noconv=False, hist_cap=4096):
        """Raises FetiError unless the solve reached its tolerance; with allow_noconv, a solve that
        stopped at the iteration cap (FETI_ENOCONV) returns its status and still writes c and dc."""
        info = feti_info()
        hist = np.zeros(hist_cap)
        info.res_hist = hist.ctypes.data_as(C.POINTER(C.c_double))
        info.res_hist_cap = hist_cap
        allow = (FETI_ENOCONV,) if allow_noconv else ()
        st = _check(lib().feti_compliance_and_grad(self.handle, _ptr(rho), _ptr(f), _ptr(c), _ptr(dc), _ptr(u),
                                                   C.byref(info)), allow=allow)
        n = min(hist_cap, info.iters + 1)
        return {"status": st, "iters": info.iters, "true_rel_res": info.true_rel_res,
                "refinements": info.refinements, "fp64_fallback": info.fp64_fallback,
                "reduced_iters": info.reduced_iters, "precision_probes": info.precision_probes,
                "reduced_rel_err": info.reduced_rel_err, "reduced_orth_err": info.reduced_orth_err,
                "history": hist[:n].copy(), "eps0": info.eps0}

    def feti_get_lambda(self, lam):
        _check(lib().feti_get_lambda(self.handle, _ptr(lam)))

    def feti_get_deflation(self, mu, Y=None):
        _check(lib().feti_get_deflation(self.handle, _ptr(mu), _ptr(Y)))

    def feti_oc_update(self, rho, dc, rho_new, volfrac, move=0.2, eta=0.5, rho_min=1e-3):
        """Returns the multiplier L of the volume bound."""
        L = C.c_double(0.0)
        _check(lib().feti_oc_update(self.handle, _ptr(rho), _ptr(dc), volfrac, move, eta, rho_min, _ptr(rho_new),
                                    C.byref(L)))
        return L.value

    def feti_apply_F(self, k, precision, Lam, Q, pure=False):
        p = PRECISIONS.get(precision, precision) | (FETI_PURE if pure else 0)
        _check(lib().feti_apply_F(self.handle, k, p, _ptr(Lam), _ptr(Q)))

    def feti_apply_F_noalloc(self, k, precision, Lam, Q, pure=False):
        p = PRECISIONS.get(precision, precision) | (FETI_PURE if pure else 0)
        _check(lib().feti_apply_F_noalloc(self.handle, k, p, _ptr(Lam), _ptr(Q)))

    def feti_apply_precond(self, r, Z, one_column, fp32=False):
        flags = int(one_column) | (FETI_PRECOND_FP32 if fp32 else 0)
        _check(lib().feti_apply_precond(self.handle, _ptr(r), _ptr(Z), flags))

    def feti_project(self, k, Y):
        _check(lib().feti_project(self.handle, k, _ptr(Y)))

    def feti_rhs(self, f, d, lambda0):
        _check(lib().feti_rhs(self.handle, _ptr(f), _ptr(d), _ptr(lambda0)))

    def feti_get_local(self, s, what):
        cap = 1 << 26
        buf = np.zeros(cap)
        r, c = C.c_int(0), C.c_int(0)
        _check(lib().feti_get_local(self.handle, s, what, buf.ctypes.data_as(C.POINTER(C.c_double)), cap,
                                    C.byref(r), C.byref(c)))
        return buf[:r.value * c.value].reshape(r.value, c.value).copy()

    def feti_autotune(self, reps=5, cache=None) -> dict:
        out = feti_tuning()
        _check(lib().feti_autotune(self.handle, reps, None if cache is None else str(cache).encode(), C.byref(out)))
        return out.as_dict()

    def feti_set_tuning(self, max_red=32, max_d=16, xcd=1, split_d=4, fp64_first=0):
        t = feti_tuning()
        t.max_red, t.max_d, t.xcd, t.split_d, t.fp64_first = max_red, max_d, xcd, split_d, fp64_first
        _check(lib().feti_set_tuning(self.handle, C.byref(t)))

    def feti_last_timing(self, what):
        ms = C.c_double(0)
        _check(lib().feti_last_timing(self.handle, what, C.byref(ms)))
        return ms.value


class BatchedContext(Context):
    """Several independent designs in one feti_ctx (feti_setup_batched): rho, f, u and the
    gradient concatenate the designs in order; the compliance has one entry per design."""

    def __init__(self, specs, rho, p=None, E0=None, Emin=None):
        if not specs:
            raise ValueError("need at least one design")
        prob = specs[0].prob
        self.spec = specs[0]
        self.specs = list(specs)
        self.p = prob.p if p is None else p
        self.E0 = prob.E0 if E0 is None else E0
        self.Emin = prob.Emin if Emin is None else Emin
        nd = len(specs)
        meshes = (feti_mesh * nd)(*[s.mesh for s in specs])
        parts = (feti_partition * nd)(*[s.part for s in specs])
        self.handle = C.c_void_p()
        _check(lib().feti_setup_batched(nd, meshes, parts, C.byref(specs[0].opts), _ptr(rho), self.p, self.E0,
                                        self.Emin, _stream(), C.byref(self.handle)))
        self.sizes = self.feti_get_sizes()
        self.layout = [self.feti_design_layout(d) for d in range(nd)]

    def feti_design_layout(self, d) -> dict:
        out = feti_design()
        _check(lib().feti_design_layout(self.handle, d, C.byref(out)))
        return out.as_dict()

    def feti_design_residuals(self) -> np.ndarray:
        out = np.zeros(len(self.specs))
        _check(lib().feti_design_residuals(self.handle, out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
        return out
