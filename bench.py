#!/usr/bin/env python3
"""Throughput of the BURA fractional solve (k+1 shifted SPD solves + FP64 combine) on one GPU.

Default workload (the batched configuration, the largest that runs on one GPU):
2D unit square, 511 x 511 interior grid, variable-coefficient five-point
operator a = exp(g) (g a seeded Gaussian random field, correlation length 0.1,
standard deviation 1, harmonic face averages) scaled to spectrum (0,1],
alpha = 0.6, beta = 1, k = 7, 256 seeded N(0,1) right-hand sides: all 8 poles x
256 right-hand sides (2048 shifted systems) advance together in the same
launches, FP32 multigrid V(2,2)-PCG inner solves with FP64 residual refinement
to relative residual 1e-10 and an FP64 combine, tile shapes chosen by the
library's tuner at plan creation.  One step = one such batched solve.

Other workloads (--workload, and the "paths" of the default line, each with
its own roofline): the 1023^2 Laplacian with alpha in {0.25, 0.5, 0.75}, k = 9,
one pole at a time in FP64 (the plain per-pole GPU solve) and batched in FP64
and mixed precision; 255^3 mixed, alpha 0.25, k = 8; the sinc quadrature,
multi-step, product and beta = 2 forms.

Prints ONE JSON line.  ``value`` counts unknown-pole solves per second
(N * (k+1) * nrhs per accepted fractional solve); a solve is accepted when its
relative l2 error against the oracle's BURA result is <= 1e-8 (checked in the
CPU-baseline leg, the only part of this script that uses the oracle).
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "unknown-pole solves/s at rel err 1e-8 vs FP64 oracle; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
HBM_TARGET_FRAC = 0.6

WORKLOADS = {
    # name: dim, n, alphas, k, nrhs, rhs kind, precision, schedule, tol, variable coefficient
    "2d1023-k9-fp64-per-pole": dict(dim=2, n=1023, alphas=(0.25, 0.5, 0.75), k=9, nrhs=1, rhs="normal", tag=2,
                                    precision="FP64", schedule="PER_POLE", tol=1e-10, var=False),
    "2d1023-k9-fp64-batched": dict(dim=2, n=1023, alphas=(0.25, 0.5, 0.75), k=9, nrhs=1, rhs="normal", tag=2,
                                   precision="FP64", schedule="BATCHED", tol=1e-10, var=False),
    "2d1023-k9-mixed-batched": dict(dim=2, n=1023, alphas=(0.25, 0.5, 0.75), k=9, nrhs=1, rhs="normal", tag=2,
                                    precision="MIXED", schedule="BATCHED", tol=1e-10, var=False),
    "2d1023-k9-fp64-multi": dict(dim=2, n=1023, alphas=(0.25, 0.5, 0.75), k=9, nrhs=1, rhs="normal", tag=2,
                                 precision="FP64", schedule="BATCHED", tol=1e-10, var=False, multi=True),
    "2d1023-k9-mixed-multi": dict(dim=2, n=1023, alphas=(0.25, 0.5, 0.75), k=9, nrhs=1, rhs="normal", tag=2,
                                  precision="MIXED", schedule="BATCHED", tol=1e-10, var=False, multi=True),
    "3d255-k8-mixed-batched": dict(dim=3, n=255, alphas=(0.25,), k=8, nrhs=1, rhs="sines", tag=3,
                                   precision="MIXED", schedule="BATCHED", tol=1e-10, var=False),
    "2d511-var-k7-256rhs-mixed": dict(dim=2, n=511, alphas=(0.6,), k=7, nrhs=256, rhs="normal", tag=4,
                                      precision="MIXED", schedule="BATCHED", tol=1e-10, var=True),
    # the sinc quadrature Section 5.3 compares against, with k_Q = 9, 7, 6 (11 + 9 + 8
    # shifted systems), on the paper's checkerboard right-hand side
    # multi-step BURA (Section 4.4): alpha = 0.75 as 0.5 then 0.25, k = 9 each (two
    # sequential stages of 10 systems); the zero-pole product form (alpha 0.5,
    # k = 9: ten sequential single-system stages)
    "2d1023-multistep-k9-fp64": dict(dim=2, n=1023, alphas=(0.5, 0.25), k=9, nrhs=1, rhs="normal", tag=2,
                                     precision="FP64", schedule="BATCHED", tol=1e-10, var=False, multi=True,
                                     method="multistep"),
    "2d1023-product-k9-fp64": dict(dim=2, n=1023, alphas=(0.5,), k=9, nrhs=1, rhs="normal", tag=2,
                                   precision="FP64", schedule="BATCHED", tol=1e-10, var=False, method="product"),
    # the 2-BURA of t^(2 - alpha) (Section 4.1), alpha 0.5, (m,k) = (7,6): 7 systems
    # together, then the chained A^-1 of the pole-0 solution
    "2d1023-beta2-k6-fp64": dict(dim=2, n=1023, alphas=(0.5,), k=6, nrhs=1, rhs="normal", tag=2,
                                 precision="FP64", schedule="BATCHED", tol=1e-12, var=False, method="beta2"),
    "2d1023-sinc-fp64-multi": dict(dim=2, n=1023, alphas=(0.25, 0.5, 0.75), k=None, kq=(9, 7, 6), nrhs=1,
                                   rhs="checkerboard", tag=0, precision="FP64", schedule="BATCHED", tol=1e-10,
                                   var=False, multi=True, method="sinc"),
}


def describe(w):
    d = w["dim"]
    grid = "x".join([str(w["n"])] * d)
    op = ("variable-coefficient a=exp(g) " if w["var"] else "") + ("5-point" if d == 2 else "7-point")
    sched = w['schedule'].lower().replace('_', '-')
    if w.get("multi"):
        sched = "batched over all poles of all alphas"
    if w.get("method") == "sinc":
        what = (f"alpha={list(w['alphas'])}, sinc quadrature (Bonito-Pasciak) with k_Q={list(w['kq'])} "
                f"applied to the unscaled operator")
    elif w.get("method") == "multistep":
        what = f"alpha={sum(w['alphas'])} as multi-step BURA steps {list(w['alphas'])}, k={w['k']} each"
        sched = "sequential steps, each step's poles batched"
    elif w.get("method") == "beta2":
        what = f"alpha={w['alphas'][0]}, beta=2, (m,k)=({w['k'] + 1},{w['k']}) 2-BURA"
        sched = "k+1 systems batched, then the chained solve"
    elif w.get("method") == "product":
        what = f"alpha={w['alphas'][0]}, beta=1, k={w['k']}, zero-pole product form"
        sched = "sequential factors"
    else:
        what = f"alpha={list(w['alphas'])}, beta=1, k={w['k']}"
    return (f"{d}D {grid} {op} operator scaled to (0,1], {what}, "
            f"{w['nrhs']} rhs ({w['rhs']}), {w['precision']} {sched} "
            f"GMG V(2,2)-PCG to rel residual {w['tol']:g}")


def make_rhs(w):
    import synth
    if w["rhs"] == "normal":
        return synth.normal_rhs(w["n"], w["dim"], nrhs=w["nrhs"], tag=w["tag"])
    if w["rhs"] == "sines":
        return synth.sine_modes_rhs(w["n"], w["dim"], nmodes=32, noise=1e-3, tag=w["tag"], nrhs=w["nrhs"])
    if w["rhs"] == "checkerboard":
        import numpy as np
        return np.repeat(synth.checkerboard_rhs(w["n"])[None], w["nrhs"], axis=0)
    return synth.uniform_rhs(w["n"], w["dim"], nrhs=w["nrhs"], tag=w["tag"])


# kernel classes timed with events in the timed region (fine-level classes, the
# FP64 refinement residual and the combine) and the ones that may be the
# roofline kernel: each covers launches of one kernel on the finest level with
# one per-point byte count (restriction and prolongation mix levels in 3D)
PROFILE_CLASSES = ("smooth_fine", "smooth_fine_rup", "down_fine", "down_fine_plain", "up_fine", "spmv",
                   "update_xr", "restrict", "prolong", "residual64", "combine")
ROOF_CLASSES = ("smooth_fine", "smooth_fine_rup", "down_fine", "down_fine_plain", "up_fine", "spmv", "update_xr",
                "residual64", "combine")
DEFAULT_WORKLOAD = "2d511-var-k7-256rhs-mixed"
DEFAULT_ALSO = ("2d1023-k9-fp64-per-pole,2d1023-k9-fp64-multi,2d1023-k9-mixed-multi,3d255-k8-mixed-batched,"
                "2d1023-sinc-fp64-multi,2d1023-multistep-k9-fp64,2d1023-product-k9-fp64,2d1023-beta2-k6-fp64")

PLAN_OPTS = {}   # plan options from --omega / --nu / --inner-tol / --autotune (empty: the library defaults)
FORCED_TILES = None   # --tiles: tile-shape variants set on each plan of the main workload


def run_gpu(w, steps, warmup, profile=True):
    import numpy as np
    import torch

    import paper_1612_04846_amd as B
    import synth

    dev = torch.device("cuda:0")
    F_host = make_rhs(w)
    F = torch.from_numpy(F_host).to(dev)
    coeff = synth.lognormal_coefficient(w["n"], w["dim"], tag=w["tag"]) if w["var"] else None
    plans = []
    t_plan = time.perf_counter()
    groups = [list(w["alphas"])] if w.get("multi") else [a for a in w["alphas"]]
    kq = {a: q for a, q in zip(w["alphas"], w.get("kq") or [None] * len(w["alphas"]))}
    for a in groups:
        kw = dict(coeff=coeff, nrhs_max=w["nrhs"], tol=w["tol"], precision=getattr(B, "BURA_" + w["precision"]),
                  schedule=getattr(B, "BURA_" + w["schedule"]), **PLAN_OPTS)
        if w.get("method") == "sinc":
            al = a if isinstance(a, list) else [a]
            kw["kprime"] = [B.sinc_kprime(x, kq[x]) for x in al]
        if w.get("method") in ("multistep", "product"):
            kw["form"] = w["method"]
        if w.get("method") == "beta2":
            kw["beta"] = 2
        plans.append(B.Plan(w["dim"], w["n"], a, w["k"], **kw))
    t_plan = time.perf_counter() - t_plan
    if FORCED_TILES is not None:
        for p, tv in zip(plans, FORCED_TILES):
            p.tiles = tv
    tiles = [p.tiles for p in plans]
    outs = [torch.empty((p.nout,) + tuple(F.shape), dtype=F.dtype, device=dev) if p.nout > 1 else torch.empty_like(F)
            for p in plans]
    for _ in range(warmup):
        for p, u in zip(plans, outs):
            p.solve(F, u)
    torch.cuda.synchronize()
    if profile:
        # events only around the fine-level kernels that can dominate (smoother or
        # fused down/up, stencil product, vector update); byte counters for all classes
        mask = sum(1 << (1 + B.KERNEL_CLASSES.index(c)) for c in PROFILE_CLASSES)
        for p in plans:
            B.bura_plan_profile(p.handle, mask)
    lat = []
    reports = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for p, u in zip(plans, outs):
            t1 = time.perf_counter()
            rep = p.solve(F, u).report
            lat.append(time.perf_counter() - t1)
            reports.append(rep)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kstats = {}
    if profile:
        for cls, name in enumerate(B.KERNEL_CLASSES):
            n_l = ms = by = 0.0
            for p in plans:
                a, b, c = B.bura_plan_kernel_stats(p.handle, cls)
                n_l += a
                ms += b
                by += c
            kstats[name] = dict(launches=int(n_l), ms=ms, bytes=by)
        for p in plans:
            B.bura_plan_profile(p.handle, False)
    info = plans[0].info
    coefs = [p.coeffs for p in plans]
    U = []
    for p, u in zip(plans, outs):
        if p.nout > 1:
            U += [u[i].cpu().numpy() for i in range(p.nout)]
        else:
            U.append(u.cpu().numpy())
    terms = [B.bura_plan_outputs(p.handle)[1][-1] for p in plans]   # shifted systems per plan and rhs
    iters = [list(r.iters)[:nt] for r, nt in zip(reports[-len(plans):], terms)]
    outer = [list(r.outer)[:nt] for r, nt in zip(reports[-len(plans):], terms)]
    relres = [max(list(r.relres)[:nt]) for r, nt in zip(reports[-len(plans):], terms)]
    for p in plans:
        p.close()
    N = w["n"] ** w["dim"]
    per_step = N * sum(terms) * w["nrhs"]
    return dict(elapsed=elapsed, per_step=per_step, lat=lat, kstats=kstats, lam=info[0], nlev=info[1],
                dev_bytes=info[2], U=U, F=F_host, coeff=coeff, coefs=coefs, iters=iters, outer=outer,
                relres=relres, t_plan=t_plan, tiles=tiles)


def roofline(kstats):
    """Dominant kernel class by event time; achieved = algorithmic bytes / event time."""
    if not kstats:
        return None, {}
    table = {}
    for name, s in kstats.items():
        if s["launches"] == 0 or s["ms"] <= 0:
            continue
        table[name] = dict(launches=s["launches"], avg_us=1e3 * s["ms"] / s["launches"],
                           alg_bytes_per_launch=s["bytes"] / s["launches"],
                           gbs=(s["bytes"] / 1e9) / (s["ms"] / 1e3) if s["bytes"] > 0 else None,
                           total_ms=s["ms"])
    cand = {k: v for k, v in table.items() if v["gbs"] is not None and k in ROOF_CLASSES}
    if not cand:
        return None, table
    dom = max(cand, key=lambda k: cand[k]["total_ms"])
    d = cand[dom]
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(d["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(d["gbs"] / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_launch_us": round(d["avg_us"], 3), "alg_bytes_per_launch": int(d["alg_bytes_per_launch"])}
    # the 60 % of HBM peak the hot path aims for; reported, not assumed
    roof["meets_hbm_target"] = roof["frac"] >= HBM_TARGET_FRAC
    return roof, table


# position of each fine-level 2D kernel class's launch shape in a plan's tiles
# (bura_plan_tiles: stencil product, then down and up per level, finest first)
TILE_INDEX = {"spmv": 0, "down_fine": 1, "down_fine_plain": 1, "up_fine": 2}


def counter_traffic(workload, kclass, tiles):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it was
    taken on the current kernel source with the same launch shape of that kernel
    (every plan of the bench line using the summary's shape; classes without
    shape variants need the same tiles throughout), else None."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1612_04846_amd", "csrc", "bura_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    idx = TILE_INDEX.get(kclass)
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_hbm_counters.md")):
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith(("#", "-", "`", " ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("workload") != workload or kv.get("kernel_class") != kclass or \
                kv.get("kernel_source_sha256_prefix") != sha:
            continue
        if idx is not None and tiles and all(len(t) > idx for t in tiles):
            same = all(str(t[idx]) == kv.get("kernel_tile") for t in tiles)
        else:
            same = kv.get("tiles") == json.dumps(tiles)
        if same:
            return int(kv["traffic_bytes_per_launch"])
    return None


def oracle_errors(w, res):
    """Relative l2 error of each GPU output against the oracle's result for the same terms."""
    from oracle import metrics, operators, quadrature, shifted, spectral
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_bura_coefficients.json")))
    errs = []
    if w.get("method") == "multistep":
        from oracle import multistep
        steps = []
        for a in w["alphas"]:
            rec = gold[f"{a:.2f},{w['k']}"]
            steps.append(([float(x) for x in rec["c"]], [float(x) for x in rec["d"]]))
        return [metrics.rel_err(res["U"][0], multistep.multistep_spectral(res["F"], w["dim"], steps))]
    if w.get("method") == "beta2":
        # 2-BURA coefficients of the oracle (multiprecision Remez, a few seconds)
        from oracle import remez as oremez
        o = oremez.remez(w["alphas"][0], w["k"], m=w["k"] + 1, beta=2)
        return [metrics.rel_err(res["U"][0], spectral.bura_beta_spectral(res["F"], w["dim"], o.c0, o.c, o.d))]
    for i, (a, U) in enumerate(zip(w["alphas"], res["U"])):
        if w.get("method") == "sinc":
            kp = quadrature.sinc_kprime(a, w["kq"][i])
            if w["var"]:
                raise ValueError("sinc workloads are constant-coefficient")
            ref = quadrature.sinc_spectral(res["F"], w["dim"], a, kp, res["lam"])
            errs.append(metrics.rel_err(U, ref))
            continue
        rec = gold[f"{a:.2f},{w['k']}"]
        c = [float(x) for x in rec["c"]]
        d = [float(x) for x in rec["d"]]
        if not w["var"]:
            ref = spectral.bura_spectral(res["F"], w["dim"], c, d)
            errs.append(metrics.rel_err(U, ref))
        else:
            # sampled right-hand sides, each by k+1 sparse direct solves
            A, _ = operators.scaled_operator(w["n"], w["dim"], res["coeff"])
            idx = [0, w["nrhs"] - 1]
            ref = shifted.bura_by_solves(A, c, d, res["F"][idx])
            errs.append(metrics.rel_err(U[idx], ref))
    return errs


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _host_info():
    return {"logical_cpus": os.cpu_count(), "cpu_model": _cpu_model(),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
            "scipy_fft_workers": os.cpu_count(),
            "superlu_threads": 1}


def exact_spectral_leg(w, F):
    """The oracle's closed-form exact A^-alpha f (DST-I, eq. (9)) on all host cores,
    median of 3: the fastest exact CPU answer for a constant-coefficient grid.
    It is not the BURA method."""
    import statistics
    import scipy.fft as sfft
    from oracle import spectral
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        with sfft.set_workers(os.cpu_count()):
            for a in w["alphas"]:
                spectral.exact_fractional(F, w["dim"], a)
        times.append(time.perf_counter() - t0)
    t = statistics.median(times)
    N = w["n"] ** w["dim"]
    return {"kind": "CPU exact spectral (not BURA)", "seconds_median_of_3": t,
            "solves_per_s": len(w["alphas"]) * w["nrhs"] / t,
            "unknowns_per_s": N * len(w["alphas"]) * w["nrhs"] / t, "cores": os.cpu_count(),
            "workload": describe(w)}


def cpu_baseline(w, res):
    """Oracle on the host: accuracy of the GPU results (every output, sampled
    right-hand sides for the variable-coefficient grid), and the timed CPU
    baseline: the oracle's k+1 shifted solves + FP64 combine as a CPU user would
    run them, on a bounded sample, median of 3, scaled to the whole workload."""
    import statistics
    import numpy as np
    from oracle import operators, shifted
    t_acc = time.perf_counter()
    errs = oracle_errors(w, res)
    t_acc = time.perf_counter() - t_acc
    N = w["n"] ** w["dim"]
    systems = res["per_step"] // (N * w["nrhs"])   # shifted systems per right-hand side and step
    if w["dim"] == 2:
        # 2D: SuperLU factorisation of one shifted system (pole d_0 = 0) and the
        # back-solves of a sample of right-hand sides; the whole workload costs
        # `systems` factorisations and systems x nrhs back-solves (the combine,
        # k+1 axpys per right-hand side, is below 0.1 % of that and left out)
        A, _ = operators.scaled_operator(w["n"], w["dim"], res["coeff"])
        rs = min(w["nrhs"], 16)
        Fs = np.ascontiguousarray(res["F"][:rs].reshape(rs, -1).T)
        tf, ts = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            lu = shifted.shifted_factor(A, 0.0)
            tf.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            lu.solve(Fs)
            ts.append((time.perf_counter() - t0) / rs)
        f_med, s_med = statistics.median(tf), statistics.median(ts)
        T = systems * f_med + systems * w["nrhs"] * s_med
        sample = dict(value=res["per_step"] / T, unit="unknown-pole solves/s", cores=1, kind="oracle",
                      sample=(f"one shifted system of the workload (pole d_0 = 0) by the oracle's SuperLU: "
                              f"factorisation, then back-solves of {rs} of its right-hand sides, each timed 3 times "
                              f"(median); scaled to the whole step ({systems} factorisations + "
                              f"{systems * w['nrhs']} back-solves = {T:.1f} s). Single-threaded: 1 of "
                              f"{os.cpu_count()} logical CPUs"),
                      factor_s_median=f_med, solve_s_per_rhs_median=s_med, factor_s_runs=tf,
                      solve_s_per_rhs_runs=ts, step_seconds_extrapolated=T, host=_host_info())
    else:
        # 3D: the oracle's plain FP64 CG on one pole of a 63^3 grid of the same
        # operator family, median of 3, scaled by unknowns (CG work per unknown
        # grows with n, so this flatters the CPU at 255^3)
        import synth
        n = 63
        A3, _ = operators.scaled_operator(n, 3)
        f = synth.normal_rhs(n, 3, tag=9).ravel()
        tc = []
        for _ in range(3):
            t0 = time.perf_counter()
            shifted.cg(A3, f, 0.0, rtol=1e-10)
            tc.append(time.perf_counter() - t0)
        dt = statistics.median(tc)
        sample = dict(value=n ** 3 / dt, unit="unknown-pole solves/s", cores=1, kind="oracle",
                      sample=f"one 63^3 shifted system (pole 0) by the oracle's plain FP64 CG to 1e-10, median of 3 "
                             f"({dt:.1f} s), single-threaded: 1 of {os.cpu_count()} logical CPUs",
                      cg_s_runs=tc, host=_host_info())
    # the closed-form exact solution on all cores, for a constant-coefficient grid
    # (the variable-coefficient workload has none: the 1023^2 Laplacian's instead)
    wex = w if not w["var"] else WORKLOADS["2d1023-k9-fp64-multi"]
    Fex = res["F"] if not w["var"] else make_rhs(wex)
    sample["exact_spectral"] = exact_spectral_leg(wex, Fex)
    return errs, sample, t_acc


def run_serving(args):
    """Seeded Poisson stream of requests through the continuous-batching server."""
    import numpy as np
    import torch

    import paper_1612_04846_amd as B
    import synth
    reqs = synth.request_stream(args.serve_requests, args.serve_rate, tag=5)
    dev = torch.device("cuda:0")
    F = [torch.from_numpy(synth.normal_rhs(r.n, r.dim, nrhs=1, tag=r.rhs_tag)[0]).to(dev) for r in reqs]
    U = [torch.empty_like(f) for f in F]
    torch.cuda.synchronize()
    budget = int(args.serve_budget_gb * (1 << 30))
    server = B.bura_server_create(budget, args.serve_concurrency, args.serve_group)

    failures = []

    def stream(timed, scale=1.0):
        """Submit every request (at its arrival time times scale when timed), wait for all."""
        t0 = time.perf_counter()
        tickets = []
        for r, f, u in zip(reqs, F, U):
            if timed:
                delay = t0 + scale * r.arrival - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            tickets.append(B.bura_server_submit(server, r.dim, r.n, r.alpha, r.k, f, u,
                                                tol=min(r.target, 1e-8), precision=B.BURA_MIXED))
        codes = []
        for i, t in enumerate(tickets):
            code, rep = B.bura_server_wait(server, t)
            codes.append(code)
            if code != B.BURA_OK:
                r = reqs[i]
                failures.append(dict(dim=r.dim, n=r.n, alpha=r.alpha, k=r.k, target=r.target, code=code,
                                     iters=list(rep.iters)[: r.k + 1], outer=list(rep.outer)[: r.k + 1],
                                     relres=[float(x) for x in list(rep.relres)[: r.k + 1]]))
            if (i + 1) % 8 == 0:
                print(f"[bench]   {i + 1}/{len(tickets)} requests done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, codes

    def per_step(b0, b1):
        """Mean number of requests sharing a solve step between two stats
        snapshots (an outer refinement step of a running solve in mixed
        precision)."""
        nb = b1["batches"] - b0["batches"]
        return (b1["mean_batch"] * b1["batches"] - b0["mean_batch"] * b0["batches"]) / nb if nb else None

    print("[bench] serving warm-up (plans and coefficients)", file=sys.stderr, flush=True)
    cold, _ = stream(False)
    cold_st = B.bura_server_stats(server)
    # latency under the Poisson arrivals, plans resident
    B.bura_server_reset_latency(server)
    print("[bench] serving timed stream (Poisson arrivals)", file=sys.stderr, flush=True)
    base = B.bura_server_stats(server)
    wall, codes = stream(True)
    st = B.bura_server_stats(server)
    # capacity: the same requests all queued at once
    print("[bench] serving capacity pass (all requests queued)", file=sys.stderr, flush=True)
    base_cap = B.bura_server_stats(server)
    wall_cap, codes_cap = stream(False)
    st_cap = B.bura_server_stats(server)
    # offered load swept around the measured capacity (arrival times rescaled)
    upole_cap = st_cap["unknown_pole_solves"] - base_cap["unknown_pole_solves"]
    cap_rate = upole_cap / wall_cap
    span = max(r.arrival for r in reqs)
    sweep = []
    for factor in args.serve_load_sweep:
        scale = upole_cap / (factor * cap_rate) / span if span > 0 else 0.0
        print(f"[bench] serving load {factor:g} x capacity", file=sys.stderr, flush=True)
        B.bura_server_reset_latency(server)
        b0 = B.bura_server_stats(server)
        w_s, codes_s = stream(True, scale)
        b1 = B.bura_server_stats(server)
        codes_cap += codes_s
        sweep.append({"load_factor": factor, "offered_solves_per_s": upole_cap / (span * scale) if scale else None,
                      "achieved_solves_per_s": (b1["unknown_pole_solves"] - b0["unknown_pole_solves"]) / w_s,
                      "p50_ms": 1e3 * b1["p50_latency_s"], "p99_ms": 1e3 * b1["p99_latency_s"],
                      "requests_per_step": per_step(b0, b1),
                      "joined_running": b1["joined_running"] - b0["joined_running"]})
    B.bura_server_destroy(server)
    ok = [c == B.BURA_OK for c in codes + codes_cap]
    upole = st["unknown_pole_solves"] - base["unknown_pole_solves"]
    return dict(wall=wall, ok=ok, stats=st, base=base, upole=upole, reqs=reqs, F=F, U=U, failures=failures,
                wall_cap=wall_cap, upole_cap=upole_cap, cold=cold, cold_p50=cold_st["p50_latency_s"],
                cold_p99=cold_st["p99_latency_s"], sweep=sweep,
                cap_batch=per_step(base_cap, st_cap))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--serving", action="store_true",
                    help="run the request-server workload (seeded Poisson stream) instead")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-rate", type=float, default=16.0, help="mean arrivals per second")
    ap.add_argument("--serve-concurrency", type=int, default=4)
    ap.add_argument("--serve-group", type=int, default=2)
    ap.add_argument("--serve-budget-gb", type=float, default=160.0)
    ap.add_argument("--serve-load-sweep", type=lambda x: [float(v) for v in x.split(",") if v],
                    default=[0.5, 0.8, 1.0, 1.2],
                    help="offered loads (multiples of the measured capacity) for the latency sweep")
    ap.add_argument("--omega", type=float, default=0.0,
                    help="uniform damping of every smoothing sweep (0: the library's default weights)")
    ap.add_argument("--nu", type=int, default=0, help="smoothing sweeps before and after (0: default 2)")
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="relative residual of the FP32 inner solves in mixed mode (0: library default)")
    ap.add_argument("--autotune", type=int, default=1, choices=(0, 1),
                    help="1: plans time the tile-shape variants at creation and keep the fastest; "
                         "0: default shapes")
    ap.add_argument("--tiles", type=json.loads, default=None,
                    help="JSON list (one list per plan) of tile-shape variants to set on the main workload's "
                         "plans after creation, e.g. the 'tiles' of an earlier bench line")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="GIB",
                    help="only run the library's streaming copy kernel over this many GiB (counter calibration)")
    ap.add_argument("--also", default=DEFAULT_ALSO,
                    help="comma-separated extra workloads reported under 'paths', each with its own roofline "
                         "(empty: none)")
    args = ap.parse_args()
    if args.omega > 0:
        PLAN_OPTS["omega"] = args.omega
    if args.nu > 0:
        PLAN_OPTS["nu_pre"] = PLAN_OPTS["nu_post"] = args.nu
    if args.inner_tol > 0:
        PLAN_OPTS["inner_tol"] = args.inner_tol
    PLAN_OPTS["autotune"] = args.autotune if args.tiles is None else 0
    if args.copy_probe > 0:
        import torch
        import paper_1612_04846_amd as B
        nbytes = int(args.copy_probe * (1 << 30))
        x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            B.bura_device_copy(y, x)
        torch.cuda.synchronize()
        # achievable rate of the library's streaming copy kernel (1 read + 1
        # write per byte), by events around 10 launches on the current stream
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(10):
            B.bura_device_copy(y, x)
        ev[1].record()
        torch.cuda.synchronize()
        t_copy = ev[0].elapsed_time(ev[1]) / 10 / 1e3
        print(json.dumps({"copy_kernel": "bura::k_stream_copy", "copy_probe_bytes_read": nbytes,
                          "copy_probe_bytes_written": nbytes, "launches": 13,
                          "copy_GBs": 2 * nbytes / t_copy / 1e9}))
        return
    if args.serving:
        res = run_serving(args)
        st = res["stats"]
        out = {"metric": METRIC, "value": None, "unit": "unknown-pole solves/s", "n_gpus": 1,
               "steps": 1, "warmup": 1, "ms_per_step": 1e3 * res["wall"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
               "data": "synthetic (seeded Poisson request stream, N(0,1) right-hand sides)",
               "config": {"workload": f"serving: {args.serve_requests} requests, Poisson rate {args.serve_rate}/s, "
                                      "grids 127^2-1023^2 and 63^3-255^3, alpha in 0.1..0.9, target 1e-6..1e-9 "
                                      "-> k 5..12, mixed precision", "max_group": args.serve_group,
                          "max_concurrent": args.serve_concurrency, "hbm_budget_gb": args.serve_budget_gb},
               "latency_ms": {"p50": 1e3 * st["p50_latency_s"], "p99": 1e3 * st["p99_latency_s"],
                              "per": "one request, submit to result, Poisson arrivals, plans resident"},
               "cold_latency_ms": {"p50": 1e3 * res["cold_p50"], "p99": 1e3 * res["cold_p99"],
                                   "per": "first pass, including plan creation (Remez, hierarchy, graphs)"},
               "offered_load_solves_per_s": res["upole"] / res["wall"],
               "capacity": {"seconds": res["wall_cap"], "unknown_pole_solves_per_s": res["upole_cap"] / res["wall_cap"],
                            "requests_per_step": res["cap_batch"], "per": "all requests queued at once"},
               "load_sweep": res["sweep"],
               "server": {k: v for k, v in st.items()}}
        accepted = all(res["ok"])
        out["failures"] = res["failures"][:12]
        if not args.no_cpu_baseline:
            # every request against the oracle's result for the same terms
            # (same alpha and k), at the metric's 1e-8; a request whose (alpha, k)
            # has no stored oracle coefficients counts as unchecked and fails
            from oracle import metrics, spectral
            gold = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_bura_coefficients.json")))
            errs, unchecked = [], 0
            for r, f, u in zip(res["reqs"], res["F"], res["U"]):
                rec = gold.get(f"{r.alpha:.2f},{r.k}")
                if not rec or "error" in rec:
                    unchecked += 1
                    accepted = False
                    continue
                ref = spectral.bura_spectral(f.cpu().numpy()[None], r.dim, [float(x) for x in rec["c"]],
                                             [float(x) for x in rec["d"]])
                e = metrics.rel_err(u.cpu().numpy()[None], ref)
                errs.append(e)
                accepted &= e <= 1e-8
            out["rel_err_vs_oracle"] = max(errs) if errs else None
            out["checked_requests"] = len(errs)
            out["unchecked_requests"] = unchecked
        out["accepted"] = accepted
        out["value"] = res["upole_cap"] / res["wall_cap"] if accepted else 0.0
        print(json.dumps(out))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    w = WORKLOADS[args.workload]
    global FORCED_TILES
    FORCED_TILES = args.tiles
    print(f"[bench] workload {args.workload}: {describe(w)}", file=sys.stderr, flush=True)
    res = run_gpu(w, args.steps, args.warmup, profile=not args.no_profile)
    import numpy as np
    lat_ms = np.array(res["lat"]) * 1e3
    roof, ktable = roofline(res["kstats"])
    if roof is not None:
        roof["traffic"] = counter_traffic(args.workload, roof["kernel"], res["tiles"])
    out = {
        "metric": METRIC,
        "value": None,
        "unit": "unknown-pole solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * res["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w["precision"] == "FP64" else "f32+f64",
        "data": "synthetic (seeded N(0,1) right-hand sides; no dataset)",
        "config": {"workload": describe(w), "name": args.workload, "dim": w["dim"], "n": w["n"],
                   "alphas": list(w["alphas"]), "k": w["k"], "nrhs": w["nrhs"], "precision": w["precision"],
                   "schedule": w["schedule"], "tol": w["tol"]},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "per": ("one solve of all alphas together" if w.get("multi") else
                               "one fractional solve (k+1 poles + combine)")},
        "iters_per_pole_last": res["iters"],
        "max_relres": max(res["relres"]),
        "lambda": res["lam"], "mg_levels": res["nlev"], "plan_seconds": round(res["t_plan"], 3),
        "tiles": res["tiles"],
        "roofline": roof,
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in ktable.items()},
    }
    raw_rate = res["per_step"] * args.steps / res["elapsed"]
    paths = {}
    FORCED_TILES = None
    for extra in [x for x in args.also.split(",") if x and x != args.workload]:
        we = WORKLOADS[extra]
        print(f"[bench] extra path {extra}", file=sys.stderr, flush=True)
        r2 = run_gpu(we, max(2, args.steps // 2), 1, profile=not args.no_profile)
        roof2, ktable2 = roofline(r2["kstats"])
        if roof2 is not None:
            roof2["traffic"] = counter_traffic(extra, roof2["kernel"], r2["tiles"])
        paths[extra] = {"workload": describe(we),
                        "value_unchecked": r2["per_step"] * max(2, args.steps // 2) / r2["elapsed"],
                        "ms_per_step": 1e3 * r2["elapsed"] / max(2, args.steps // 2),
                        "dtype": "f64" if we["precision"] == "FP64" else "f32+f64",
                        "iters_per_pole_last": r2["iters"], "outer_last": r2["outer"], "tiles": r2["tiles"],
                        "roofline": roof2,
                        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                                    for k, v in ktable2.items()},
                        "_res": r2, "_w": we}
    accepted = True
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        errs, sample, t_acc = cpu_baseline(w, res)
        out["rel_err_vs_oracle"] = max(errs)
        accepted = max(errs) <= 1e-8
        out["cpu_baseline"] = sample
        for name, pth in paths.items():
            ee = oracle_errors(pth["_w"], pth["_res"])
            pth["rel_err_vs_oracle"] = max(ee)
            pth["value"] = pth["value_unchecked"] if max(ee) <= 1e-8 else 0.0
    else:
        out["rel_err_vs_oracle"] = None
        out["cpu_baseline"] = None
    for pth in paths.values():
        pth.pop("_res", None)
        pth.pop("_w", None)
    out["value"] = raw_rate if accepted else 0.0
    out["accepted"] = accepted
    out["paths"] = paths
    print(json.dumps(out))


if __name__ == "__main__":
    main()
