"""Benchmark: complete FEAST solves per second on one MI355X.

One step = one full feast_solve (factor all Ne shifted systems, refinement
loops to convergence, residuals) on the tight-binding chain workload
(nc=2000 cells of b=64, n=128000, M0=128, Ne=8, interval holding 80
eigenvalues), inputs resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload tb128k] [--no-extra]
                  [--precision 0|1|2] [--graph 0|1|2] [--no-cpu-baseline]

--workload tbbatch times feast_solve_batched on the first --batch uneven
problems of the batched workload (each step solves all of them);
--workload tbbatch256 on all 256 problems of its full shape (nc up to 500,
b up to 96).

--graph 1 passes the graph option of feast_solve (loops after the first
replay one captured HIP graph) to every solve of the batched workload.

--workload htb32k times feast_solve_hermitian (eq. 12) on a complex chain of
the tb32k shape (nc=500, b=64, n=32000, M0=64, Ne=8, 38 eigenvalues).

--precision 1 times the mixed-precision solver instead (factor blocks rounded
to float32, complex float32 sweeps, float64 refinement of every shifted solve
to a relative residual of 1e-12); --precision 2 float32 solves in the first
loop only.

The default run (tb128k, float64) adds four legs to the same JSON line:
"mixed" (the mixed-precision solver on the same workload, with its gate
against the stored oracle result and its time relative to float64),
"adaptive" (float32 solves in the first loop only), "batched" (the 256
uneven problems of the full batched shape, Ne = 16, solved together) and
"hermitian" (the htb32k solve above), each with its own gate and roofline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The batched legs drive one HIP stream per host worker (16); HIP maps a
# process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 by default).
# Measured: 32-problem batch 480 problems/s with 8 workers on 4 queues, 557
# on 8, 575 on 16; the 256-problem batch 106 with 8 workers on 8 queues and
# 151 with 16 on 16.  Set before the HIP runtime starts.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")

METRIC = "FEAST solves/sec and shifted-solve TFLOP/s (% MFMA peak) at 1e-10 eig accuracy"
PEAK_FP64 = 78.6        # TFLOP/s, MI355X dense FP64 (matrix = vector)
PEAK_FP32 = 157.3       # TFLOP/s, MI355X dense FP32 (matrix = vector)
PEAK_HBM = 8000.0       # GB/s


# sources the shifted-solve kernels (factorisation, sweeps) are built from
SOLVE_SOURCES = ("common.h", "kernels.h", "factor.hip", "sweep.hip")


def source_digest(names=SOLVE_SOURCES):
    """Digest of the shifted-solve kernel sources: HBM traffic taken with
    counters applies only to kernels built from exactly these sources."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0901_2665_amd", "csrc")
    for name in sorted(names):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None
    when the summary is missing or the sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    digest, value = None, None
    for line in open(path):
        if line.startswith("source digest:"):
            digest = line.split(":", 1)[1].strip()
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 2 and cells[0] == kernel:
            try:
                value = float(cells[-1])
            except ValueError:
                pass
    if digest != source_digest():
        return None
    return value


def copy_probe():
    """A plain device copy of 1 GiB (read 1 GiB, write 1 GiB): the reference
    that scales the HBM byte counters."""
    import torch
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def nominal_flops(nc, b, m0, ne):
    """Nominal work of the sequential block-LU algorithm (complex = 4x real)."""
    d = dict(
        factor=ne * nc * (56.0 / 3.0) * b ** 3,          # per solve
        forward_sweep=ne * nc * 16.0 * b * b * m0,        # per loop: W^T h and Sinv h
        back_sweep=ne * nc * 8.0 * b * b * m0,            # per loop: W x
        # mixed precision, per launch: the same sweeps in float32, and the
        # float64 residual R - (Z_e B - A) x_e of all nodes (A and B times
        # the real and imaginary planes: 4 block-tridiagonal products)
        refine_residual=ne * nc * 24.0 * b * b * m0,
    )
    d["forward_sweep32"] = d["forward_sweep"]
    d["back_sweep32"] = d["back_sweep"]
    return d


def host_cpu():
    """Model and core counts of the host that runs the oracle."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(p, emin, emax, m0, ne, Y0, loops):
    """Time the oracle on a bounded sample of the same workload: one shifted
    factorisation, one shifted solve with all M0 right-hand sides, one
    projection + reduced eigensolve + Ritz vectors; extrapolate to a full
    solve with Ne shifts and the GPU's loop count.  The factorisation and
    the solve are timed again on one thread (16 right-hand sides, scaled)."""
    from oracle import feast_oracle as O
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max(i["num_threads"] for i in threadpool_info())
    except Exception:
        threadpool_limits = None
        threads = 1
    ct = O.contour(emin, emax, ne)
    t0 = time.perf_counter()
    lu = O.factor_shift(p, ct.Z[0])
    t1 = time.perf_counter()
    R = O.assemble(p.Bd, p.Bu) @ Y0
    Qe = lu.solve(R)
    t2 = time.perf_counter()
    Q = np.real(Qe)
    AQ, BQ = O.project(p, Q)
    eps, Phi, _ = O.reduced_eig(AQ, BQ)
    _ = Q @ Phi
    t3 = time.perf_counter()
    t_factor, t_solve, t_rr = t1 - t0, t2 - t1, t3 - t2
    t_full = ne * t_factor + loops * (ne * t_solve + t_rr)
    out = {"value": 1.0 / t_full, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
           "sample": (f"1 banded LU factorisation ({t_factor:.1f}s) + 1 solve with {m0} "
                      f"right-hand sides ({t_solve:.1f}s) + 1 projection/Rayleigh-Ritz "
                      f"({t_rr:.1f}s) of the same workload, extrapolated to {ne} shifts x "
                      f"{loops} loops = {t_full:.0f}s per solve"),
           "host": host_cpu()}
    if threadpool_limits is not None:
        k = min(16, m0)
        with threadpool_limits(limits=1):
            s0 = time.perf_counter()
            lu1 = O.factor_shift(p, ct.Z[0])
            s1 = time.perf_counter()
            lu1.solve(R[:, :k])
            s2 = time.perf_counter()
        f1, v1 = s1 - s0, (s2 - s1) * m0 / k
        t1_full = ne * f1 + loops * (ne * v1 + t_rr)
        out["single_thread"] = {
            "value": 1.0 / t1_full, "unit": "solves/s", "cores": 1,
            "sample": (f"1 factorisation ({f1:.1f}s) + 1 solve with {k} right-hand sides "
                       f"scaled to {m0} ({v1:.1f}s) on one thread; the projection/Rayleigh-"
                       f"Ritz time of the multi-thread sample; extrapolated as above = "
                       f"{t1_full:.0f}s per solve")}
    return out


def solve_leg(ctx, workload, precision, steps, warmup, cpu=True, graph=0):
    """Timed complete solves of one workload; returns the bench-line fields."""
    import torch
    from paper_0901_2665_amd import feast as F
    from paper_0901_2665_amd import workloads as W
    p, emin, emax, m0, ne, Y0 = W.make_workload(workload)
    wl = W.WORKLOADS[workload]
    gp = F.Pencil(p.Ad, p.Au, p.Bd, p.Bu)
    y = torch.as_tensor(Y0, dtype=torch.float64, device="cuda").contiguous()
    out = (torch.empty(m0, dtype=torch.float64, device="cuda"),
           torch.empty((p.n, m0), dtype=torch.float64, device="cuda"),
           torch.empty(m0, dtype=torch.float64, device="cuda"))
    prec = precision
    for _ in range(warmup):
        r = ctx.solve(gp, emin, emax, m0, ne, y, out=out, precision=prec, graph=graph)
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.perf_counter()
    results = []
    for _ in range(steps):
        r = ctx.solve(gp, emin, emax, m0, ne, y, out=out, precision=prec, graph=graph)
        results.append((r.status, r.M, r.loops, r.max_res))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    times = ctx.timing_read()
    ctx.timing(False)
    elapsed = t1 - t0

    # accuracy gate on the last solve
    lam = out[0].cpu().numpy()
    gate = {"M": r.M, "expected_M": wl["n_eig"], "max_res": r.max_res, "loops": r.loops,
            "status": r.status, "rr_sweeps": r.rr_sweeps}
    if prec == 1:
        gate["refine_steps"] = r.refine_steps
        gate["shifted_solve_rel_res"] = r.solve_res
    gpath = os.path.join(ROOT, "tests", "golden", f"feast_{workload}.json")
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        ref = np.array(g["lam"])
        if len(ref) == r.M:
            gate["max_rel_eig_err_vs_oracle"] = float(np.max(np.abs(lam[:r.M] - ref) / np.abs(ref)))
        gate["oracle_loops"] = g["loops"]
        gate["oracle_max_res"] = g["max_res"]
    gate["pass"] = bool(r.M == wl["n_eig"] and r.max_res <= 1e-9 and r.status == 0 and
                        gate.get("max_rel_eig_err_vs_oracle", 0.0) <= 1e-10 and
                        all(s_ == 0 and M == r.M for s_, M, _, _ in results))

    nom = nominal_flops(p.nc, p.b, m0, ne)
    per = {}
    for k, (ms, cnt) in times.items():
        if cnt:
            per[k] = {"ms_total": ms, "launches": cnt, "ms_avg": ms / cnt}
    if prec == 1:
        solve_kernels = ["factor", "round_factors", "forward_sweep32", "back_sweep32",
                         "refine_residual"]
        peak_of = {"forward_sweep32": PEAK_FP32, "back_sweep32": PEAK_FP32}
    elif prec == 2:
        solve_kernels = ["factor", "round_factors", "forward_sweep32", "back_sweep32",
                         "forward_sweep", "back_sweep"]
        peak_of = {"forward_sweep32": PEAK_FP32, "back_sweep32": PEAK_FP32}
    else:
        solve_kernels = ["factor", "forward_sweep", "back_sweep"]
        peak_of = {}
    dom = max((k for k in solve_kernels if k in nom), key=lambda k: times.get(k, (0, 0))[0])
    ms_dom, n_dom = times[dom]
    achieved = nom[dom] / (ms_dom / n_dom * 1e-3) / 1e12
    peak_dom = peak_of.get(dom, PEAK_FP64)
    loops_total = sum(x[2] for x in results)
    shifted_ms = sum(times[k][0] for k in solve_kernels if k in times)
    shifted_flops = steps * nom["factor"] + loops_total * (nom["forward_sweep"] +
                                                          nom["back_sweep"])
    shifted_tflops = shifted_flops / (shifted_ms * 1e-3) / 1e12
    shifted_peak = PEAK_FP32 if prec == 1 else PEAK_FP64
    leg = {
        "value": steps / elapsed,
        "unit": "solves/s",
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * elapsed / steps,
        "dtype": "f32+f64" if prec in (1, 2) else "f64",
        "config": {"workload": workload, "nc": p.nc, "b": p.b, "n": p.n, "M0": m0,
                   "Ne": ne, "interval": [emin, emax], "eigenvalues_in_interval": wl["n_eig"],
                   "tol": 1e-12,
                   "precision": {0: "float64", 1: "mixed", 2: "adaptive"}[prec],
                   "graph": graph},
        "shifted_solve_tflops": shifted_tflops,
        "shifted_solve_frac_peak": shifted_tflops / shifted_peak,
        "gate": gate,
        "kernels": per,
        "roofline": {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": peak_dom,
                     "unit": "TFLOP/s", "frac": achieved / peak_dom,
                     "traffic": (measured_traffic(workload, dom) if prec == 0 else None)},
    }
    if cpu:
        leg["cpu_baseline"] = cpu_baseline(p, emin, emax, m0, ne, Y0, r.loops)
    return leg


def hermitian_cpu_baseline(p, emin, emax, m0, ne, Y0, loops):
    """The Hermitian oracle on a bounded sample of the same workload: one
    banded LU of Z_1 B - A, both solves of eq. 12 with all M0 right-hand
    sides, one projection + reduced eigensolve; extrapolated to Ne shifts and
    the GPU's loop count."""
    from oracle import feast_oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max(i["num_threads"] for i in threadpool_info())
    except Exception:
        threads = 1
    ct = O.contour(emin, emax, ne)
    t0 = time.perf_counter()
    lu = O.factor_shift_hermitian(p, ct.Z[0])
    t1 = time.perf_counter()
    R = O.assemble(p.Bd, p.Bu) @ Y0
    x = lu.solve(R)
    y = lu.solve(R, adjoint=True)
    t2 = time.perf_counter()
    AQ, BQ = O.project_hermitian(p, x + y)
    eps, Phi, _ = O.reduced_eig_hermitian(AQ, BQ)
    _ = (x + y) @ Phi
    t3 = time.perf_counter()
    t_factor, t_solve, t_rr = t1 - t0, t2 - t1, t3 - t2
    t_full = ne * t_factor + loops * (ne * t_solve + t_rr)
    return {"value": 1.0 / t_full, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"1 complex banded LU ({t_factor:.1f}s) + the solve and the adjoint "
                       f"solve with {m0} right-hand sides ({t_solve:.1f}s) + 1 projection/"
                       f"Rayleigh-Ritz ({t_rr:.1f}s) of the same workload, extrapolated to "
                       f"{ne} shifts x {loops} loops = {t_full:.0f}s per solve"),
            "host": host_cpu()}


def hermitian_leg(ctx, steps, warmup, cpu=True, workload="htb32k"):
    """Complete solves of the Hermitian variant (eq. 12) on a complex chain of
    the tb32k shape; gated against the eigenvalues that the oracle's inertia
    bisection stored with the interval."""
    import torch
    from paper_0901_2665_amd import feast as F
    from paper_0901_2665_amd import workloads as W
    p, emin, emax, m0, ne, Y0 = W.make_workload(workload)
    wl = W.WORKLOADS[workload]
    hp = F.HermitianPencil(p.Ad, p.Au, p.Bd, p.Bu)
    y = torch.as_tensor(np.ascontiguousarray(Y0), dtype=torch.complex128, device="cuda")
    for _ in range(warmup):
        r = ctx.solve_hermitian(hp, emin, emax, m0, ne, y)
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.perf_counter()
    results = []
    for _ in range(steps):
        r = ctx.solve_hermitian(hp, emin, emax, m0, ne, y)
        results.append((r.status, r.M))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    times = ctx.timing_read()
    ctx.timing(False)
    ref = np.array(json.load(open(os.path.join(ROOT, "tests", "golden", "intervals.json")))
                   [workload]["eigenvalues"])
    lam = r.lam.cpu().numpy()[:r.M]
    scale = np.maximum(np.abs(ref), 0.5 * (emax - emin))
    err = float(np.max(np.abs(lam - ref) / scale)) if r.M == len(ref) else None
    gate = {"M": r.M, "expected_M": wl["n_eig"], "max_res": r.max_res, "loops": r.loops,
            "status": r.status, "max_rel_eig_err_vs_bisection": err}
    gate["pass"] = bool(r.M == wl["n_eig"] and r.status == 0 and r.max_res <= 1e-9 and
                        err is not None and err <= 1e-10 and
                        all(s_ == 0 and M == r.M for s_, M in results))
    # nominal work: block LU of a non-symmetric complex block-tridiagonal
    # matrix per contour point (LU of S_i, W_i, V_i, S_{i+1}: (8/3 + 24) b^3
    # real flops a cell); per loop both solves of eq. 12, each a forward
    # (Sinv h, V h) and a back (W x) block product per cell
    nom = {"factor": ne * p.nc * (80.0 / 3.0) * p.b ** 3,
           "sweeps_hermitian": ne * p.nc * 48.0 * p.b * p.b * m0}
    per = {k: {"ms_total": ms, "launches": c, "ms_avg": ms / c} for k, (ms, c) in times.items()
           if c}
    dom = max(nom, key=lambda k: times.get(k, (0, 0))[0])
    ms_dom, n_dom = times[dom]
    achieved = nom[dom] / (ms_dom / n_dom * 1e-3) / 1e12
    leg = {"value": steps / elapsed, "unit": "solves/s", "steps": steps, "warmup": warmup,
           "ms_per_step": 1e3 * elapsed / steps, "dtype": "c128",
           "config": {"workload": workload, "nc": p.nc, "b": p.b, "n": p.n, "M0": m0, "Ne": ne,
                      "interval": [emin, emax], "eigenvalues_in_interval": wl["n_eig"],
                      "tol": 1e-12, "variant": "hermitian (eq. 12)"},
           "gate": gate, "kernels": per,
           "roofline": {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None}}
    if cpu:
        leg["cpu_baseline"] = hermitian_cpu_baseline(p, emin, emax, m0, ne, Y0, r.loops)
    return leg


def batch_leg(ctx, count, precision, steps, warmup, workers=0, graph=0, cpu=True,
              workload="tbbatch"):
    """Independent uneven problems solved together by feast_solve_batched;
    value = problems solved per second.  tbbatch: nc 50..200, b 32/48/64;
    tbbatch256: the full shape, 256 problems, nc 50..500, b 32/64/96 (b = 96
    on the generic kernels); M0 16..64 and Ne 16 for both."""
    import torch
    from paper_0901_2665_amd import feast as F
    from paper_0901_2665_amd import workloads as W
    if workload == "tbbatch256":
        probs = W.make_batch256(count)
        shape_of = W.batch256_shape
    else:
        probs = W.make_batch(count)
        shape_of = W.batch_shape
    dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").contiguous()
    batch = [(F.Pencil(p.Ad, p.Au, p.Bd, p.Bu), emin, emax, m0, ne, dev(Y0))
             for p, emin, emax, m0, ne, Y0 in probs]
    tol = 1e-13  # the paper's trace tolerance (Sec. IV.A)
    for _ in range(warmup):
        ctx.solve_batched(batch, tol=tol, precision=precision, workers=workers, graph=graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st, rs = ctx.solve_batched(batch, tol=tol, precision=precision, workers=workers,
                                   graph=graph)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    want = [shape_of(i)["n_eig"] for i in range(count)]
    # status 2 (B_Q fallback: with Ne = 16 the filtered outside directions
    # can vanish numerically) still writes converged outputs
    gate = {"status": st, "statuses": sorted({r.status for r in rs}),
            "all_M_match": all(r.M == m for r, m in zip(rs, want)),
            "max_res": max(r.max_res for r in rs), "loops_max": max(r.loops for r in rs),
            "above_1e-9": [i for i, r in enumerate(rs) if r.max_res > 1e-9]}
    gate["pass"] = bool(all(r.status in (0, 2) for r in rs) and gate["all_M_match"] and
                        gate["max_res"] <= 1e-9)
    shapes = [shape_of(i) for i in range(count)]
    # whole-step rate: nominal shifted-solve work of every problem (factor once,
    # forward and back sweeps per loop) over the wall time of the step
    flops = 0.0
    for s_, r in zip(shapes, rs):
        nom = nominal_flops(s_["nc"], s_["b"], s_["M0"], s_["Ne"])
        flops += nom["factor"] + r.loops * (nom["forward_sweep"] + nom["back_sweep"])
    achieved = flops * steps / elapsed / 1e12
    leg = {
        "value": steps * count / elapsed,
        "unit": "problems/s",
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * elapsed / steps,
        "dtype": "f32+f64" if precision == 1 else "f64",
        "config": {"workload": workload, "problems": count,
                   "nc": [min(x["nc"] for x in shapes), max(x["nc"] for x in shapes)],
                   "b": sorted({x["b"] for x in shapes}),
                   "M0": [min(x["M0"] for x in shapes), max(x["M0"] for x in shapes)],
                   "Ne": W.BATCH_NE, "tol": tol,
                   "precision": "mixed" if precision == 1 else "float64",
                   "workers": workers or min(count, 8), "graph": graph},
        "gate": gate,
        # kernels of the workers' streams are not timed one by one: the
        # nominal shifted-solve work of the whole step over its wall time
        "roofline": {"bound": "mfma", "kernel": "whole batched step (shifted solves, nominal)",
                     "achieved": achieved,
                     "peak": PEAK_FP32 if precision == 1 else PEAK_FP64, "unit": "TFLOP/s",
                     "frac": achieved / (PEAK_FP32 if precision == 1 else PEAK_FP64),
                     "traffic": None},
    }
    if cpu:
        leg["cpu_baseline"] = batch_cpu_baseline(probs, shapes, [r.loops for r in rs])
    return leg


def batch_cpu_baseline(probs, shapes, loops):
    """The oracle's complete FEAST solve of the batch problem with the least
    nominal work, extrapolated to the batch by the nominal shifted-solve work
    of each problem."""
    from oracle import feast_oracle as O
    work = lambda s_, lp: (nominal_flops(s_["nc"], s_["b"], s_["M0"], s_["Ne"])["factor"] +
                           lp * sum(nominal_flops(s_["nc"], s_["b"], s_["M0"], s_["Ne"])[k]
                                    for k in ("forward_sweep", "back_sweep")))
    i0 = min(range(len(shapes)), key=lambda i: work(shapes[i], loops[i]))
    p, emin, emax, m0, ne, Y0 = probs[i0]
    t0 = time.perf_counter()
    r = O.feast(p, emin, emax, m0, ne, Y0, tol=1e-13)
    t = time.perf_counter() - t0
    scale = sum(work(s_, lp) for s_, lp in zip(shapes, loops)) / work(shapes[i0], r.loops)
    s0 = shapes[i0]
    return {"value": len(shapes) / (t * scale), "unit": "problems/s", "kind": "oracle",
            "cores": host_cpu()["usable_cpus"], "extrapolated": True,
            "sample": (f"complete oracle solve of problem {i0} (nc {s0['nc']}, b {s0['b']}, "
                       f"M0 {s0['M0']}: {t:.1f}s, {r.loops} loops), extrapolated to the "
                       f"{len(shapes)} problems by nominal work (x{scale:.1f})")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tb128k")
    ap.add_argument("--precision", type=int, default=0, choices=(0, 1, 2),
                    help="0: float64 shifted solves; 1: mixed precision; 2: float32 "
                         "solves in the first loop only (experiment)")
    ap.add_argument("--batch", type=int, default=32,
                    help="problems per step of the tbbatch workload")
    ap.add_argument("--workers", type=int, default=16,
                    help="host workers (HIP streams) of the batched workloads; 0 = the "
                         "library's default (8)")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1, 2),
                    help="1 = loops after the first replay a captured HIP graph; 2 = the "
                         "convergence decision on the device, four loops per graph launch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline line (no mixed-precision and batched legs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU FEAST "
              "hot path; multi-GPU sharding is described in DESIGN.md, not run.",
              file=sys.stderr)
        sys.exit(2)

    from paper_0901_2665_amd import feast as F

    if args.copy_probe:
        copy_probe()
    ctx = F.Context(0)
    cpu = not args.no_cpu_baseline
    if args.workload in ("tbbatch", "tbbatch256"):
        count = args.batch if args.workload == "tbbatch" else 256
        leg = batch_leg(ctx, count, args.precision, args.steps, args.warmup, args.workers,
                        args.graph, cpu, workload=args.workload)
    elif args.workload == "htb32k":
        leg = hermitian_leg(ctx, args.steps, args.warmup, cpu)
    else:
        leg = solve_leg(ctx, args.workload, args.precision, args.steps, args.warmup, cpu,
                        graph=args.graph)
    line = {"metric": METRIC, "value": leg.pop("value"), "unit": leg.pop("unit"), "n_gpus": 1}
    line.update({k: leg.pop(k) for k in ("steps", "warmup", "ms_per_step")})
    line.update({"higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                 "dtype": leg.pop("dtype"), "data": "synthetic"})
    line.update(leg)
    print(f"bench: {args.workload} leg done ({line['value']:.2f} {line['unit']})", file=sys.stderr,
          flush=True)
    if args.workload == "tb128k" and args.precision == 0 and not args.no_extra:
        # the scope table's next rows on the same box, same run: mixed precision
        # on the same workload, and the batched uneven problems
        mixed = solve_leg(ctx, "tb128k", 1, 2, 1, cpu=False)
        mixed["vs_float64"] = mixed["value"] / line["value"]
        if cpu:
            mixed["cpu_baseline"] = dict(line["cpu_baseline"], extrapolated=True,
                                         note="the float64 oracle of the headline line")
        line["mixed"] = mixed
        print(f"bench: mixed leg done ({mixed['value']:.2f} solves/s)", file=sys.stderr, flush=True)
        # labelled experiment: float32 solves in the first loop only, float64 after
        adaptive = solve_leg(ctx, "tb128k", 2, 2, 1, cpu=False)
        adaptive["vs_float64"] = adaptive["value"] / line["value"]
        line["adaptive"] = adaptive
        print(f"bench: adaptive leg done ({adaptive['value']:.2f} solves/s)", file=sys.stderr,
              flush=True)
        # two warm-up steps: every worker's workspace reaches the largest
        # problem it meets before the timed steps
        line["batched"] = batch_leg(ctx, 256, 0, 2, 2, workers=args.workers, cpu=cpu,
                                    workload="tbbatch256")
        print(f"bench: batched leg done ({line['batched']['value']:.1f} problems/s)",
              file=sys.stderr, flush=True)
        line["hermitian"] = hermitian_leg(ctx, 2, 1, cpu=cpu)
        print(f"bench: hermitian leg done ({line['hermitian']['value']:.2f} solves/s)",
              file=sys.stderr, flush=True)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
