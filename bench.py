#!/usr/bin/env python
"""Benchmark of the FETI hot path on one MI355X.

Metric: FETI-DP solve time to a relative residual of 1e-6 (S-FETI-DP with k-scaling and
64 simultaneous directions) with F*Lambda in FP32 on the matrix cores, next to the plain
FP64 form, plus F*Lambda GFLOP/s in FP64, FP32 and split BF16.

Workload: 2D Q4 plane stress, 16 x 16 subdomains of 64 x 64 elements (2 101 250 DOFs),
rho ~ Beta(0.3, 0.3) per element (seed 0), E0 = 1, Emin = 1e-9, p = 3, nu = 0.3, left edge
clamped, unit load at right-mid; subdomains grouped in 2 x 2 blocks for 64 directions.

One step = feti_compliance_and_grad(rho, f): assembly, factorisation and explicit local
operators (setup), the Krylov solve to 1e-6, recovery of u, compliance and its gradient.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 157.3}   # TFLOP/s of the comparable dense peak
HBM_PEAK_GBS = 8000.0


def flambda_work(sizes, k):
    """Algorithmic flops of one whole F*Lambda: local products Y_s = F_s X_s and T_s = F_rc^sT X_s,
    the coarse solve and the fold Y_s += F_rc^s v (2k sum n_b^2 + 4k sum n_b n_c + 2k n_cg^2)."""
    flops = 2.0 * k * sizes["sum_nb2"] + 4.0 * k * sizes["sum_nb_nc"] + 2.0 * k * sizes["n_cg"] ** 2
    return flops


def flambda_kernel_split(sizes, k):
    """Algorithmic flops of the local-product kernel alone, split by the matrix cores that run
    them in the in-solve (hybrid) form: F_s X_s of the subdomains that keep the reduced precision
    on FP32 MFMA; F_s X_s of the subdomains that failed the round-off test and every T_s = F_rc^sT X_s
    on FP64 MFMA. Returns (fp32 flops, fp64 flops)."""
    f64 = 2.0 * k * (sizes["sum_nb2_fp64"] + sizes["sum_nb_nc"])
    f32 = 2.0 * k * (sizes["sum_nb2"] - sizes["sum_nb2_fp64"])
    return f32, f64


def hybrid_peak(f32, f64):
    """Peak of a kernel that runs f32 flops on the FP32 and f64 flops on the FP64 matrix cores,
    one after the other on the same CUs: total flops over the sum of the two times at peak."""
    return (f32 + f64) / (f32 / PEAK["fp32"] + f64 / PEAK["fp64"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


ROOF_KERNEL = "k_flambda<1, 4, double>"  # in-solve F*Lambda, 64 directions: FP32 rows + FP64 rows, FP64 outputs
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "flambda_insolve_c3_traffic.json")
COPY_BYTES = 1 << 30                     # calibration copy for the HBM byte counters


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("k_apply.hip", "kernels.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2111_11728_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch of the roofline kernel from the committed rocprofv3 counter runs,
    or None when the kernel sources changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("traffic_bytes_per_launch")


def ingest_pmc(fetch_dir, write_dir):
    """Turn two rocprofv3 --pmc runs of `bench.py --flambda-only` (FETCH_SIZE, WRITE_SIZE; KiB
    per dispatch) into the traffic record: each counter is scaled by what it reads for the plain
    device copy of COPY_BYTES in the same run."""
    import glob
    import sqlite3

    def per_kernel(d, counter):
        dbs = glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)
        if not dbs:
            raise SystemExit(f"no rocpd database under {d}")
        con = sqlite3.connect(dbs[0])
        rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection").fetchall()
        out = {}
        for disp, name, cname, val in rows:
            if cname != counter:
                continue
            out.setdefault(name, []).append((int(disp), float(val)))
        return out

    f = per_kernel(fetch_dir, "FETCH_SIZE")
    w = per_kernel(write_dir, "WRITE_SIZE")

    def pick(tab, key, largest=False, last=None):
        vals = sorted(v for n, vs in tab.items() if key in n for v in vs)
        if last:
            vals = vals[-last:]
        vals = [v for _, v in vals]
        if not vals:
            raise SystemExit(f"kernel {key} not in counter run")
        return float(max(vals) if largest else np.median(vals))

    # the calibration copies are the largest device copies of the run; the roofline kernel's
    # launches on the tile shapes the autotuner chose are its last eight (3 warm-up + 5 timed)
    cf, cw = pick(f, "copyBuffer", True), pick(w, "copyBuffer", True)
    kf, kw = pick(f, ROOF_KERNEL, last=8), pick(w, ROOF_KERNEL, last=8)
    sf, sw = COPY_BYTES / (cf * 1024.0), COPY_BYTES / (cw * 1024.0)
    rec = {"kernel": ROOF_KERNEL, "source_hash": kernel_source_hash(),
           "fetch_kib_per_launch": kf, "write_kib_per_launch": kw,
           "copy_fetch_kib": cf, "copy_write_kib": cw, "scale_fetch": sf, "scale_write": sw,
           "traffic_bytes_per_launch": kf * 1024.0 * sf + kw * 1024.0 * sw}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


GOLDEN = os.path.join(ROOT, "tests", "golden")


def errors_vs_oracle(u, c, g, dirs):
    """Errors of one GPU solve against the oracle's stored records of the same workload (files
    written by scripts that call only the oracle): u at the 4096 sampled DOFs against the global
    direct solution and against the oracle's own S-FETI-DP solve at the same tolerance, relative
    to the norm of the whole vector; the compliance and the gradient at 20 sampled elements
    against the oracle's. Empty when the records are absent."""
    out = {}
    try:
        star = np.load(os.path.join(GOLDEN, "c3_u_sample.npz"))
        us = u.cpu().numpy()[star["idx"]]
        out["u_vs_direct"] = float(np.linalg.norm(us - star["u"]) / star["norm"])
    except OSError:
        pass
    try:
        rec = np.load(os.path.join(GOLDEN, "c3_sfeti.npz"))
        key = f"k{dirs}_"
        us = u.cpu().numpy()[rec["idx"]]
        out["u_vs_oracle_sfeti"] = float(np.linalg.norm(us - rec[key + "u"]) / rec[key + "u_norm"])
        out["c_vs_oracle_sfeti"] = abs(c - float(rec[key + "c"])) / abs(float(rec[key + "c"]))
        ge = g.cpu().numpy()[rec["el_idx"]]
        out["g_vs_oracle_sfeti"] = float(np.linalg.norm(ge - rec[key + "g"]) / np.linalg.norm(rec[key + "g"]))
        out["oracle_iters"] = int(rec[key + "iters"])
    except (OSError, KeyError):
        pass
    return out


def cpu_baseline(dirs):
    """The oracle (plain CPU FP64) on this workload, on the host cores of this machine.

    The oracle cannot run the full workload inside a benchmark (its setup alone takes minutes), so
    the full-size run is a stored record: tests/golden/c3_sfeti.npz holds the oracle's setup and
    S-FETI-DP solve seconds at full size (2 101 250 DOFs), measured by the script that wrote it,
    together with that machine's CPU and thread count. Here the bounded sample of the same design
    that the record's machine also timed (tests/golden/c3_cpu_sample.json: setup and 12 iterations
    on the 4x4-subdomain block, workloads.beta_2d_block) is timed again on this host, and the
    full-size record is carried over by the ratio of the two sample times."""
    import workloads
    from oracle import feti as ofeti
    from oracle import krylov as okrylov
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    runs = []
    for _ in range(2):
        sub = workloads.beta_2d_block(0)
        t0 = time.perf_counter()
        op = ofeti.FETIDP(sub, "dirichlet", "k")
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        res = okrylov.simultaneous(op, tol=1e-6, max_it=12)
        runs.append((t_setup, time.perf_counter() - t0, res.iters))
    t_setup, t_solve = min(r[0] for r in runs), min(r[1] for r in runs)
    out = {"unit": "ms", "cores": int(threads), "kind": "oracle"}
    try:
        rec = np.load(os.path.join(GOLDEN, "c3_sfeti.npz"))
        with open(os.path.join(GOLDEN, "c3_cpu_sample.json")) as fh:
            cal = json.load(fh)
    except (OSError, ValueError):
        out.update(value=None, sample=f"sample only (no stored full-size record): setup {t_setup:.2f} s, "
                                       f"{runs[0][2]} iterations in {t_solve:.2f} s")
        return out
    ratio_solve, ratio_setup = t_solve / cal["solve_s"], t_setup / cal["setup_s"]
    key = f"k{dirs}_"
    full_solve, full_setup = float(rec[key + "t_solve"]), float(rec["t_setup"])
    out.update(
        value=1e3 * full_solve * ratio_solve, setup_ms=1e3 * full_setup * ratio_setup,
        oracle_iters=int(rec[key + "iters"]),
        full_size_record={"solve_s": full_solve, "setup_s": full_setup, "iters": int(rec[key + "iters"]),
                          "cpu": str(rec["cpu_model"]), "threads": int(rec["threads"])},
        sample=(f"oracle S-FETI-DP (k-scaling, Dirichlet) at full size is a stored record ({full_solve:.0f} s solve, "
                f"{full_setup:.0f} s setup, {int(rec[key + 'iters'])} iterations, {int(rec['threads'])} threads of "
                f"{rec['cpu_model']}); the bounded sample (setup and 12 iterations on the 4x4-subdomain block "
                f"of the same design) took {t_setup:.2f} s + {t_solve:.2f} s here against {cal['setup_s']:.2f} s + "
                f"{cal['solve_s']:.2f} s there; value = record solve time x sample solve-time ratio "
                f"({ratio_solve:.2f})"))
    return out


def run_c4(args):
    """Batched workload: independent uneven 2D designs (gx, gy ~ U{4..8} subdomains, widths and
    heights ~ U{16..48} elements, modular 0/1 densities, seed 0) in one batched context, S-FETI-DP
    with k-scaling, each design with one direction per subdomain; one step = compliance and
    gradient of every design. Prints its own JSON line (not the headline metric)."""
    import torch

    import workloads
    from paper_2111_11728_amd import feti

    dev = torch.device("cuda:0")
    probs = [workloads.uneven_design(0, d) for d in range(args.c4_designs)]
    specs = [feti.Spec(pr, method="fetidp", scaling="k", krylov="sfeti", precond="dirichlet",
                       precision=args.c4_precision, tol=args.tol, max_it=args.max_it) for pr in probs]
    rho = torch.tensor(np.concatenate([pr.rho for pr in probs]), device=dev)
    f = torch.tensor(np.concatenate([pr.load() for pr in probs]), device=dev)
    t0 = time.perf_counter()
    cx = feti.BatchedContext(specs, rho)
    torch.cuda.synchronize()
    log(f"batched setup: {time.perf_counter() - t0:.2f} s, {cx.sizes['n_sub']} subdomains, "
        f"{cx.sizes['device_bytes'] / 2**30:.1f} GiB")
    nd = len(probs)
    c = torch.zeros(nd, dtype=torch.float64, device=dev)
    g = torch.zeros(sum(pr.n_el for pr in probs), dtype=torch.float64, device=dev)
    u = torch.zeros(sum(pr.n_dof for pr in probs), dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        cx.feti_compliance_and_grad(rho, f, c, g, u)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        info = cx.feti_compliance_and_grad(rho, f, c, g, u)
        rec.append((cx.feti_last_timing(2), cx.feti_last_timing(3), info))
        log(f"c4 step {i}: setup {rec[-1][0]:.1f} ms, solve {rec[-1][1]:.1f} ms, {info['iters']} iterations, "
            f"worst design true rel. residual {info['true_rel_res']:.2e}")
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / max(1, args.steps)
    res_d = cx.feti_design_residuals()
    line = {"metric": f"batched solve time, {nd} independent uneven designs (S-FETI-DP, k-scaling, one direction "
                      f"per subdomain of each design, tol {args.tol})",
            "value": float(np.mean([r[1] for r in rec])), "unit": "ms", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": wall, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if args.c4_precision == "fp64" else "f32+f64", "data": "synthetic",
            "config": {"workload": f"{nd} uneven 2D modular designs (4-8 x 4-8 subdomains of 16-48 elements, seed 0)",
                       "n_sub": cx.sizes["n_sub"], "n_dof": cx.sizes["n_dof"], "n_lambda": cx.sizes["n_lambda"],
                       "n_cg": cx.sizes["n_cg"], "directions": cx.sizes["n_groups"]},
            "setup_ms": float(np.mean([r[0] for r in rec])), "iters": rec[-1][2]["iters"],
            "worst_design_true_rel_res": float(res_d.max()), "compliance_sum": float(c.sum())}
    cx.close()
    print(json.dumps(line))


def run_c5(args):
    """3D workload: Hex8 elasticity on 4x4x4 subdomains of 12^3 elements, seeded 0/1 modular
    density, contrast 1e-6; S-FETI-DP with k-scaling and the Dirichlet preconditioner, F*Lambda
    mixed FP32/FP64 (--c5-precision fp64 for the plain form); one step = compliance and gradient
    (setup, solve, recovery, adjoint). Also times F*Lambda at k = 64 in FP64 and FP32. Prints its
    own JSON line (not the headline metric)."""
    import torch

    import workloads
    from paper_2111_11728_amd import feti

    dev = torch.device("cuda:0")
    prob = workloads.modular_3d(0)
    spec = feti.Spec(prob, method="fetidp", scaling="k", krylov="sfeti", precond="dirichlet",
                     precision=args.c5_precision, tol=args.tol, max_it=args.max_it)
    rho = torch.tensor(prob.rho, device=dev)
    f = torch.tensor(prob.load(), device=dev)
    t0 = time.perf_counter()
    cx = feti.Context(spec, rho)
    torch.cuda.synchronize()
    log(f"c5 setup: {time.perf_counter() - t0:.2f} s, n_lambda {cx.sizes['n_lambda']}, "
        f"{cx.sizes['n_fp64_subs']} subdomains kept in FP64")
    fl = {}
    k = 64
    L = torch.randn(cx.sizes["n_lambda"], k, device=dev, dtype=torch.float64)
    Q = torch.zeros_like(L)
    for prec in ("fp64", "fp32"):
        for _ in range(3):
            cx.feti_apply_F(k, prec, L, Q, pure=True)
        ts = []
        for _ in range(args.flambda_reps):
            cx.feti_apply_F(k, prec, L, Q, pure=True)
            ts.append(cx.feti_last_timing(0))
        fl[prec] = float(np.mean(ts)) * 1e3
        log(f"c5 F*Lambda {prec}, k = {k}: kernel {fl[prec]:.1f} us (default tile shapes)")
    # tile shapes of the in-solve F*Lambda chosen on the device for the solve (no cache: tuned
    # every run); they apply to every tile list, so the pure-precision timings above come first
    tune = cx.feti_autotune(reps=3)
    log(f"c5 autotune: max_red {tune['max_red']}, max_d {tune['max_d']}, xcd {tune['xcd']}, split_d {tune['split_d']}: "
        f"{tune['us']:.1f} us (default shapes {tune['us_default']:.1f} us)")
    c = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(prob.n_el, dtype=torch.float64, device=dev)
    u = torch.zeros(prob.n_dof, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        cx.feti_compliance_and_grad(rho, f, c, g, u)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        info = cx.feti_compliance_and_grad(rho, f, c, g, u)
        rec.append((cx.feti_last_timing(2), cx.feti_last_timing(3), info))
        log(f"c5 step {i}: setup {rec[-1][0]:.1f} ms, solve {rec[-1][1]:.1f} ms, {info['iters']} iterations "
            f"({info['reduced_iters']} reduced), true rel. residual {info['true_rel_res']:.2e}")
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / max(1, args.steps)
    line = {"metric": f"3D FETI-DP solve time to rel.res {args.tol} (S-FETI, k-scaling)",
            "value": float(np.mean([r[1] for r in rec])), "unit": "ms", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": wall, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if args.c5_precision == "fp64" else "f32+f64", "data": "synthetic",
            "config": {"workload": "3D Hex8, 4x4x4 subdomains of 12^3 elements, modular 0/1 rho, contrast 1e-6",
                       "n_dof": prob.n_dof, "n_lambda": cx.sizes["n_lambda"], "n_cg": cx.sizes["n_cg"],
                       "directions": cx.sizes["n_groups"]},
            "setup_ms": float(np.mean([r[0] for r in rec])), "iters": rec[-1][2]["iters"],
            "reduced_iters": rec[-1][2]["reduced_iters"], "true_rel_res": rec[-1][2]["true_rel_res"],
            "flambda_k64_us": fl, "tuning": tune, "compliance": float(c.item())}
    cx.close()
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dirs", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--flambda-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp64-solve", action="store_true")
    ap.add_argument("--orth-fp32", action="store_true",
                    help="opt-in: FP32 Gram-Schmidt against the stored directions on reduced iterations")
    ap.add_argument("--precond-fp64", action="store_true",
                    help="mixed solve: the preconditioner from its FP64 blocks (default: FP32 copies)")
    ap.add_argument("--max-it", type=int, default=1000)
    ap.add_argument("--flambda-only", action="store_true",
                    help="only the F*Lambda microbenchmark and a calibration copy (for counter runs)")
    ap.add_argument("--ingest-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic record from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--c4", action="store_true", help="the batched multi-design workload instead of the headline")
    ap.add_argument("--c4-designs", type=int, default=64)
    ap.add_argument("--c4-precision", default="fp64")
    ap.add_argument("--c5", action="store_true", help="the 3D workload instead of the headline")
    ap.add_argument("--c5-precision", default="fp32")
    args = ap.parse_args()
    if args.ingest_pmc:
        ingest_pmc(*args.ingest_pmc)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): it measures one GPU's share of the "
              f"subdomains at its real shape; sharding them over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    if args.c4:
        run_c4(args)
        return
    if args.c5:
        run_c5(args)
        return

    import torch

    import workloads
    from paper_2111_11728_amd import feti

    dev = torch.device("cuda:0")
    prob = workloads.beta_2d(0, n_dirs=args.dirs)
    rho = torch.tensor(prob.rho, device=dev)
    f = torch.tensor(prob.load(), device=dev)

    def make(precision):
        spec = feti.Spec(prob, method="fetidp", scaling="k", krylov="sfeti", precond="dirichlet",
                         precision=precision, tol=args.tol, max_it=args.max_it, orth_fp32=int(args.orth_fp32),
                         precond_fp32=int(precision != "fp64" and not args.precond_fp64))
        t0 = time.perf_counter()
        cx = feti.Context(spec, rho)
        log(f"setup {precision}: {time.perf_counter() - t0:.2f} s, {cx.sizes['device_bytes'] / 2**30:.1f} GiB")
        return cx

    out = {}
    ctx = make("fp32")
    sizes = ctx.sizes
    n_l = sizes["n_lambda"]
    # ---- F*Lambda microbenchmark (k = 64 directions) ----
    k = 64
    gen = torch.Generator(device=dev).manual_seed(0)
    L = torch.randn(n_l, k, generator=gen, device=dev, dtype=torch.float64)
    Q = torch.zeros_like(L)
    flops = flambda_work(sizes, k)
    fl = {}
    # pure: every row block in the named precision (the kernel rate, on the default tile shapes);
    # "fp32_solve": the form the mixed solve applies (FP32 where the round-off test allows, FP64
    # F_rc^T rows and the rest), on the shapes the autotuner then picks for it
    tune = None
    for name, prec, pure in [("fp64", "fp64", True), ("fp32", "fp32", True), ("bf16x3", "bf16x3", True),
                             ("fp32_solve", "fp32", False)]:
        if not pure and tune is None:
            # tile shapes of the in-solve F*Lambda chosen on the device (no cache: tuned every run);
            # they apply to every tile list, so the pure-precision timings come first
            tune = ctx.feti_autotune(reps=5)
            log(f"autotune: max_red {tune['max_red']}, max_d {tune['max_d']}, xcd {tune['xcd']}, "
                f"split_d {tune['split_d']}: {tune['us']:.1f} us (default shapes {tune['us_default']:.1f} us)")
        for _ in range(3):
            ctx.feti_apply_F(k, prec, L, Q, pure=pure)
        kern, tot = [], []
        for _ in range(args.flambda_reps):
            ctx.feti_apply_F(k, prec, L, Q, pure=pure)
            kern.append(ctx.feti_last_timing(0))
            tot.append(ctx.feti_last_timing(1))
        km, tm = float(np.mean(kern)), float(np.mean(tot))
        log(f"F*Lambda {name}: kernel {1e3 * km:.1f} us, total {1e3 * tm:.1f} us")
        elem = 8 if prec == "fp64" else 4
        bytes_ = elem * sizes["sum_nb2"] + 2 * 8 * n_l * k
        fl[name] = {"kernel_us": 1e3 * km, "total_us": 1e3 * tm,
                    "gflops_kernel": flops / (km * 1e-3) / 1e9, "gflops_total": flops / (tm * 1e-3) / 1e9,
                    "frac_peak_kernel": flops / (km * 1e-3) / 1e12 / PEAK[prec],
                    "hbm_gbs_kernel": bytes_ / (km * 1e-3) / 1e9}
    out["flambda"] = fl
    if args.flambda_only:
        src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"flambda": fl}))
        return

    # ---- full steps ----
    c = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.zeros(prob.n_el, dtype=torch.float64, device=dev)
    u = torch.zeros(prob.n_dof, dtype=torch.float64, device=dev)

    def run_steps(cx, nwarm, nsteps):
        for _ in range(nwarm):
            cx.feti_compliance_and_grad(rho, f, c, g, u)
        torch.cuda.synchronize()
        rec = []
        t0 = time.perf_counter()
        for i in range(nsteps):
            info = cx.feti_compliance_and_grad(rho, f, c, g, u)
            rec.append((cx.feti_last_timing(2), cx.feti_last_timing(3), info))
            log(f"step {i}: setup {rec[-1][0]:.1f} ms, solve {rec[-1][1]:.1f} ms, {info['iters']} iterations, "
                f"true rel. residual {info['true_rel_res']:.2e}, fp64 fallback {info['fp64_fallback']}, "
                f"reduced {info['reduced_iters']}, eta {info['reduced_rel_err']:.2e} "
                f"(orth {info['reduced_orth_err']:.2e})")
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / max(1, nsteps)
        return wall, rec

    wall_m, rec_m = run_steps(ctx, args.warmup, args.steps)
    u_m = u.clone()
    g_m = g.clone()
    c_m = float(c.item())
    vs_oracle = {"mixed": errors_vs_oracle(u_m, c_m, g_m, args.dirs)}
    solve_m = float(np.mean([r[1] for r in rec_m]))
    setup_m = float(np.mean([r[0] for r in rec_m]))
    info_m = rec_m[-1][2]
    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    res64 = {}
    if not args.skip_fp64_solve:
        ctx64 = make("fp64")
        wall_d, rec_d = run_steps(ctx64, args.warmup, args.steps)
        res64 = {"solve_ms": float(np.mean([r[1] for r in rec_d])), "step_ms": wall_d,
                 "iters": rec_d[-1][2]["iters"], "true_rel_res": rec_d[-1][2]["true_rel_res"],
                 "u_rel_diff_mixed_vs_fp64": float(torch.linalg.norm(u - u_m) / torch.linalg.norm(u)),
                 "compliance_rel_diff": abs(float(c.item()) - c_m) / abs(float(c.item())),
                 "grad_rel_diff_mixed_vs_fp64": float(torch.linalg.norm(g - g_m) / torch.linalg.norm(g))}
        vs_oracle["fp64"] = errors_vs_oracle(u, float(c.item()), g, args.dirs)
        ctx64.close()
        del ctx64
        torch.cuda.empty_cache()
        # an FP64 solve to tol 1e-10 (untimed): the error that each timed solve keeps at its own
        # tolerance, over the whole of u and g (the two solves stop at the same preconditioned
        # residual along different search spaces, so their difference is of the size of that error)
        spec_t = feti.Spec(prob, method="fetidp", scaling="k", krylov="sfeti", precond="dirichlet",
                           precision="fp64", tol=1e-10, max_it=args.max_it)
        ctx_t = feti.Context(spec_t, rho)
        u_t = torch.zeros_like(u)
        g_t = torch.zeros_like(g)
        c_t = torch.zeros_like(c)
        info_t = ctx_t.feti_compliance_and_grad(rho, f, c_t, g_t, u_t)
        ctx_t.close()
        nu_t, ng_t = torch.linalg.norm(u_t), torch.linalg.norm(g_t)
        res64["vs_fp64_tol1e-10"] = {
            "iters": info_t["iters"],
            "u_err_mixed": float(torch.linalg.norm(u_m - u_t) / nu_t),
            "u_err_fp64": float(torch.linalg.norm(u - u_t) / nu_t),
            "g_err_mixed": float(torch.linalg.norm(g_m - g_t) / ng_t),
            "g_err_fp64": float(torch.linalg.norm(g - g_t) / ng_t)}

    gpu_iters = info_m["iters"]
    # roofline of the dominant kernel of the timed solve: the in-solve F*Lambda local products
    f32, f64 = flambda_kernel_split(sizes, k)
    pk = hybrid_peak(f32, f64)
    ins = fl["fp32_solve"]
    ach = (f32 + f64) / (ins["kernel_us"] * 1e-6) / 1e12
    whole = flops / (ins["total_us"] * 1e-6) / 1e12
    roof = {"bound": "mfma", "achieved": ach, "peak": pk, "unit": "TFLOP/s", "frac": ach / pk,
            "traffic": load_traffic(),
            "kernel": ROOF_KERNEL + " (in-solve F*Lambda local products, k = 64: F_s X_s on FP32 MFMA, "
                      "T_s = F_rc^sT X_s and the subdomains that failed the round-off test on FP64 MFMA)",
            "flops_per_launch": f32 + f64, "flops_fp32": f32, "flops_fp64": f64,
            "peak_fp32": PEAK["fp32"], "peak_fp64": PEAK["fp64"], "avg_launch_us": ins["kernel_us"],
            "whole_apply": {"flops": flops, "avg_us": ins["total_us"], "achieved": whole, "frac": whole / pk,
                            "what": "gather, local products, coarse correction, fold and scatter (one F*Lambda)"},
            "pure_fp32": {"kernel": "k_flambda<1, 4, float> (microbenchmark: every row block FP32, FP32 outputs)",
                          "achieved": 2.0 * k * (sizes["sum_nb2"] + sizes["sum_nb_nc"]) / (fl["fp32"]["kernel_us"] * 1e-6)
                          / 1e12, "peak": PEAK["fp32"], "avg_launch_us": fl["fp32"]["kernel_us"]}}
    roof["pure_fp32"]["frac"] = roof["pure_fp32"]["achieved"] / PEAK["fp32"]
    line = {
        "metric": "FETI-DP solve time to rel.res 1e-6 (S-FETI-DP, k-scaling, 64 directions, FP32 F*Lambda); "
                  "F*Lambda GFLOP/s mixed vs FP64",
        "value": solve_m, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall_m, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "beta2d_16x16_of_64x64: 2D Q4, 16x16 subdomains of 64x64 elements, "
                               "rho~Beta(0.3,0.3) seed 0, Emin/E0=1e-9, p=3",
                   "n_dof": prob.n_dof, "n_lambda": n_l, "n_cg": sizes["n_cg"], "directions": sizes["n_groups"],
                   "tol": args.tol},
        "setup_ms": setup_m, "iters": gpu_iters, "refinements": info_m["refinements"],
        "fp64_fallback": info_m["fp64_fallback"], "reduced_iters": info_m["reduced_iters"],
        "precision_probes": info_m["precision_probes"], "reduced_rel_err": info_m["reduced_rel_err"],
        "reduced_orth_err": info_m["reduced_orth_err"], "orth_fp32": int(args.orth_fp32),
        "precond_fp32": int(not args.precond_fp64),
        "true_rel_res": info_m["true_rel_res"], "fp64": res64,
        "flambda": fl, "roofline": roof, "autotune": tune, "vs_oracle": vs_oracle,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle: bounded sample here, carried over to the stored full-size record)")
        line["cpu_baseline"] = cpu_baseline(args.dirs)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
