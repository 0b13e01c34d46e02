#!/usr/bin/env python3
"""Throughput of the fracsolve hot path on one MI355X.

A step is one full solve (right-hand-side assembly, every leaf and every
level product) of one synthetic instance already resident in HBM.  Default
workload: time-fractional diffusion, gamma = 0.3, M = 4096 interior points,
N = 65536 time steps, manufactured t^2 sin(pi x) source plus 8 seeded random
modes a_j t^p_j sin(j pi x), float64.  The printed value is M*N unknowns per
second over the timed steps.  The error is checked against the oracle
through single-mode reduction (every source mode's discrete solution is
v_j^n sin(j pi x_i), with v_j from the oracle's scalar recurrence).

roofline: the FFT level products (the HBM-bound part of the path), every
level, single-pass and multi-pass, timed live with HIP events around each
launch on the solver's stream during one extra solve; achieved = their
algorithmic bytes (24 B per X-row entry: read X, read and write Y) / their
summed time, against the 8 TB/s HBM peak, with each level's own figure and
the worst level listed.  critical_path: the sequential chain of leaf solves (one workgroup
per launch, two leaves per launch where they run in pairs), which sets most
of the solve time.
forms (unless --no-forms): mixed precision and the variant with the spatial
term averaged over t_n and t_{n-1} (c3), batching (c4), the adjoint (c5) and
the paper's own iterative method, restarted GMRES(m), on its
Example 4 meshes next to the recursive solve (--config gmres runs only that;
with --N 2^k only the mesh h = tau = 2^-k), and the advection equations
(Schemes 2 and 3) on the paper's timing meshes (--config advection), and
Scheme 1, the two-sided fractional ODE by FFT conjugate gradients, on the
meshes of its timing table (--config ode; with --N 2^k only that mesh).
cpu_baseline: the oracle (plain time stepping) on the same workload for the
first --cpu-steps steps at full width; its wall time is scaled to the full
run, by the ratio measured once for this workload on the GPU host
(bench.py --cpu-full, recorded in profiles/) where there is one, otherwise by
(N / steps)^2 (the history work is quadratic in the step count), and
reported as unknowns per second.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "M·N unknowns solved/sec at stated err vs FP64 oracle; mixed/batched vs plain FP64"
HBM_PEAK_GBS = 8000.0

# single-pass FFT kernel instantiations (k_fft.hip): n -> template text
FFT64_NAMES = {
    8: "k_fft2u<double, 4, 2, 8, true>", 16: "k_fft2u<double, 4, 4, 8, true>",
    32: "k_fft2u<double, 8, 4, 8, true>", 64: "k_fft2u<double, 8, 8, 8, true>",
    128: "k_fft2u<double, 16, 8, 8, true>", 256: "k_fft2u<double, 16, 16, 8, true>",
    512: "k_fft3u<double, 16, 8, 4, 8, 256, true>", 1024: "k_fft3u<double, 16, 8, 8, 8, 256, true>",
    2048: "k_fft3u<double, 16, 16, 8, 4, 256, true>", 4096: "k_fft3u<double, 16, 16, 16, 2, 256, true>",
    8192: "k_fft3u<double, 16, 16, 32, 1, 256, true>",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def recorded_traffic(s: int, M: int):
    """HBM bytes per level product of half-size s (every kernel of that level:
    the transform kernel, with the near-corner band kernel where the band has
    one, or the three multi-pass kernels) recorded in profiles/ (FETCH_SIZE and WRITE_SIZE passes scaled by
    the copy calibration), or None when there is no record for this M or the
    FFT source changed since it was taken."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "fft_level_traffic_M%d.md" % M)
    src = os.path.join(ROOT, "paper_1710_11593_amd", "csrc", "k_fft.hip")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for line in open(path):
        m = re.match(r'traffic: s=(\d+) bytes_per_launch=(\d+) k_fft_sha=(\w+)', line.strip())
        if m and int(m.group(1)) == s and m.group(3) == sha:
            return float(m.group(2))
    return None


def recorded_full_run(config: str, M: int, N: int, gamma: float, n_s: int):
    """The whole-run oracle time recorded in profiles/ for this workload
    (bench.py --cpu-full on the GPU host), or None."""
    import re

    path = os.path.join(ROOT, "profiles", "oracle_c2_full_run.md")
    if config != "c2" or n_s != 8192 or not os.path.exists(path):
        return None
    for line in open(path):
        m = re.match(r"full_run: workload=c2 M=(\d+) N=(\d+) gamma=([\d.]+) threads=(\d+) total_s=([\d.]+) "
                     r"first_8192_s=([\d.]+)$", line.strip())
        if m and int(m.group(1)) == M and int(m.group(2)) == N and abs(float(m.group(3)) - gamma) < 1e-12:
            return {"threads": int(m.group(4)), "total_s": float(m.group(5)), "first_s": float(m.group(6))}
    return None


def fft_roofline(ks, prec, M):
    """Roofline of the FFT level products (the HBM-bound part of the path):
    every FFT level of the solve, single-pass and multi-pass, from the
    per-launch event times of one solve.  achieved = their algorithmic bytes
    (24 B per X-row entry and launch: read X, read and write Y) / their summed
    time, against the 8 TB/s HBM peak; the near-corner band launches that
    complete the single-pass levels count in the time.  levels lists each
    level's own figure; worst names the slowest."""
    fft_kind = "fft_f64" if prec == "fp64" else "fft_f32"
    lv = [g for g in ks if g["kind"] == fft_kind and g["ms"] > 0]
    if not lv:
        return None
    corner = {g["s"]: g for g in ks if g["kind"] == "fft_corner"}
    levels = []
    for g in sorted(lv, key=lambda r: r["s"]):
        ms = g["ms"] + (corner[g["s"]]["ms"] if g["s"] in corner else 0.0)
        levels.append({"s": g["s"], "launches": g["launches"], "ms": round(ms, 4),
                       "GBps": round(g["bytes"] / (ms * 1e-3) / 1e9, 1),
                       "frac": round(g["bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    tot_b = sum(g["bytes"] for g in lv)
    tot_ms = sum(l["ms"] for l in levels)
    achieved = tot_b / (tot_ms * 1e-3) / 1e9
    worst = min(levels, key=lambda l: l["frac"])
    big = max(lv, key=lambda r: r["s"])
    kname = ("fs::" + FFT64_NAMES[2 * big["s"]]) if (prec == "fp64" and 2 * big["s"] in FFT64_NAMES) else None
    traffic = None
    if prec == "fp64":
        # recorded HBM bytes of every level over their algorithmic bytes
        rec = [(recorded_traffic(g["s"], M), g) for g in lv]
        if rec and all(r is not None for r, _ in rec):
            traffic = sum(r * g["launches"] for r, g in rec)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "FFT level products, all levels (s = %d .. %d), time-weighted" % (levels[0]["s"],
                                                                                      levels[-1]["s"]),
            "algorithmic_bytes": tot_b, "ms": round(tot_ms, 3), "worst_level": worst, "levels": levels,
            "largest_single_pass_kernel": kname}


FP64_MFMA_PEAK_TFS = 78.6


def mfma_levels(ks, M, mfma_from=128):
    """Matrix-core utilisation of the dense level products that run on the
    float64 MFMA kernel (half-size s >= mfma_from): executed flops 2 s^2 M
    per launch (a full block; the last block of a solve can be shorter) over
    their event-timed duration, against the 78.6 TF/s float64 matrix peak."""
    out = []
    for g in sorted(ks, key=lambda r: r["s"]):
        if g["kind"] != "dense_f64" or g["s"] < mfma_from or g["ms"] <= 0:
            continue
        fl = 2.0 * g["s"] * g["s"] * M * g["launches"]
        tf = fl / (g["ms"] * 1e-3) / 1e12
        out.append({"s": g["s"], "launches": g["launches"], "ms": round(g["ms"], 4), "TFLOPs": round(tf, 2),
                    "frac": round(tf / FP64_MFMA_PEAK_TFS, 4)})
    return out


def build_instance(args):
    from paper_1710_11593_amd import workloads as wl

    if args.config == "c2":
        gamma = args.gamma if args.gamma else 0.3
        inst = wl.c2(gamma=gamma, seed=3 if gamma == 0.7 else 2, M=args.M or 4096, N=args.N or 65536,
                     build=False)
        desc = "diffusion gamma=%g, M=%d, N=%d, manufactured t^2 sin(pi x) + 8 seeded modes" % (
            inst.gamma, inst.M, inst.N)
    elif args.config == "c3":
        inst = wl.c3(M=args.M or 2048, N=args.N or 131072, build=False)
        desc = "diffusion-wave gamma=1.5, M=%d, N=%d, u=(t^2+1) sin(pi x)" % (inst.M, inst.N)
    elif args.config == "c1":
        inst = wl.c1()
        inst.f = None
        desc = "diffusion gamma=0.5, M=64, N=256, u=t^2 sin(pi x)"
    else:
        raise SystemExit("unknown --config %s" % args.config)
    return inst, desc


def modal_factors(inst):
    """(js, G [N][k], u0 coefficient per mode, phi coefficient per mode)."""
    import numpy as np

    from paper_1710_11593_amd import workloads as wl

    series = wl.modal_time_series(inst)
    js = sorted(series)
    G = np.stack([series[j][0] for j in js], axis=1)
    return js, G, [series[j][1] for j in js], [series[j][2] for j in js]


def device_inputs(inst, dev):
    """f = G S (built on the device), u0, phi and the modal factors of inst."""
    import numpy as np
    import torch

    from paper_1710_11593_amd import workloads as wl

    js, G, c_u0, c_phi = modal_factors(inst)
    x, _, _, _ = wl.grid(inst.M, inst.N)
    S = np.stack([np.sin(j * math.pi * x) for j in js])
    Sd = torch.from_numpy(S).to(dev)
    f = (torch.from_numpy(G).to(dev) @ Sd).contiguous()
    u0 = torch.from_numpy(np.asarray(c_u0) @ S).to(dev)
    phi = torch.from_numpy(np.asarray(c_phi) @ S).to(dev)
    return dict(f=f, u0=u0, phi=phi, js=js, G=G, c_u0=c_u0, c_phi=c_phi, Sd=Sd)


def mode_error(inst, d, u, threads=16, cn=False):
    """Max-norm relative error of u against the oracle through single-mode
    reduction (each source mode's discrete solution from the oracle's scalar
    recurrence; cn: of the variant with the spatial term averaged over t_n
    and t_{n-1})."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import oracle
    from paper_1710_11593_amd import workloads as wl

    key = "Vcn" if cn else "V"
    if key not in d:  # the oracle's modal time series, computed once per instance
        _, _, h, _ = wl.grid(inst.M, inst.N)
        js, G = d["js"], d["G"]
        lam = [4.0 / h ** 2 * math.sin(j * math.pi * h / 2) ** 2 for j in js]
        mode = oracle.mode_cn if cn else oracle.mode
        with ThreadPoolExecutor(max_workers=min(threads, len(js))) as ex:
            vs = list(ex.map(lambda k: mode(inst.gamma, inst.T, inst.N, lam[k], G[:, k], d["c_u0"][k],
                                            d["c_phi"][k]), range(len(js))))
        d[key] = torch.from_numpy(np.stack(vs, axis=1)).to(u.device)
    ref = d[key] @ d["Sd"]
    return float((u - ref).abs().max() / ref.abs().max())


def timed(fn, reps):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def run_forms(dev):
    """The other forms of the metric, each against the plain float64 GPU solve
    of the same instances: c2 at gamma = 0.7, mixed precision (c3), batching
    (c4) and the adjoint (c5).  Returns a dict for the JSON line."""
    import numpy as np
    import torch

    from paper_1710_11593_amd import binding, workloads as wl

    out = {}
    # c2 at its second stated gamma (0.7; the headline line runs gamma = 0.3)
    inst = wl.c2(gamma=0.7, seed=3, build=False)
    d = device_inputs(inst, dev)
    u = torch.empty_like(d["f"])
    sv = binding.Solver([dict(gamma=inst.gamma, M=inst.M, N=inst.N)])
    run = lambda: sv.solve([d["f"]], [d["u0"]], out=[u])  # noqa: E731
    run()
    ms = timed(run, 3)
    err = mode_error(inst, d, u)
    sv.close()
    out["c2_gamma0.7_fp64"] = {"ms": round(ms, 2), "unknowns_per_s": inst.M * inst.N / (ms * 1e-3),
                               "error_vs_oracle": err}
    log("forms: c2 gamma 0.7 fp64 %.1f ms, err %.3e" % (ms, err))
    del d, u
    torch.cuda.empty_cache()
    # c3: diffusion-wave, float64 vs float32 products + one refinement step
    inst = wl.c3(build=False)
    d = device_inputs(inst, dev)
    u = torch.empty_like(d["f"])
    res = {}
    for prec, ref in (("fp64", 0), ("fp32", 1)):
        sv = binding.Solver([dict(gamma=inst.gamma, M=inst.M, N=inst.N)], precision=prec, refine_steps=ref)
        run = lambda: sv.solve([d["f"]], [d["u0"]], [d["phi"]], out=[u])  # noqa: E731
        run()
        ms = timed(run, 2)
        err = mode_error(inst, d, u)
        res[prec] = {"ms": round(ms, 2), "unknowns_per_s": inst.M * inst.N / (ms * 1e-3), "error_vs_oracle": err,
                     "refine_steps": ref}
        sv.close()
        log("forms: c3 %s %.1f ms, err %.3e" % (prec, ms, err))
    out["c3_mixed_fp32"] = res["fp32"]
    out["c3_fp64"] = res["fp64"]
    out["mixed_speedup_vs_fp64"] = round(res["fp64"]["ms"] / res["fp32"]["ms"], 3)
    # the same workload with the spatial term averaged over t_n and t_{n-1}
    sv = binding.Solver([dict(gamma=inst.gamma, M=inst.M, N=inst.N)], equation="diffusion_cn")
    run = lambda: sv.solve([d["f"]], [d["u0"]], [d["phi"]], out=[u])  # noqa: E731
    run()
    ms = timed(run, 2)
    err = mode_error(inst, d, u, cn=True)
    sv.close()
    out["c3_averaged_spatial_term_fp64"] = {"ms": round(ms, 2), "unknowns_per_s": inst.M * inst.N / (ms * 1e-3),
                                            "error_vs_oracle": err}
    log("forms: c3 averaged spatial term fp64 %.1f ms, err %.3e" % (ms, err))
    del d, u
    torch.cuda.empty_cache()

    # c4: 256 uneven instances, one batched handle (float32 + refinement) vs
    # the same instances one by one in float64
    insts = wl.c4()
    ds = [device_inputs(i, dev) for i in insts]
    us = [torch.empty_like(x["f"]) for x in ds]
    probs = [dict(gamma=i.gamma, M=i.M, N=i.N) for i in insts]
    wave = [i.gamma > 1 for i in insts]
    sample = list(range(0, len(insts), 32))
    batched = {}
    for prec, ref in (("fp64", 0), ("fp32", 1)):
        sb = binding.Solver(probs, precision=prec, refine_steps=ref)
        run = lambda: sb.solve([x["f"] for x in ds], [x["u0"] for x in ds],  # noqa: E731
                               [x["phi"] if w else None for x, w in zip(ds, wave)], out=us)
        run()
        ms_b = timed(run, 1)
        sb.close()
        batched[prec] = (ms_b, max(mode_error(insts[k], ds[k], us[k]) for k in sample))
    solvers = [binding.Solver([p]) for p in probs]

    def one_by_one():
        for k, sv in enumerate(solvers):
            sv.solve([ds[k]["f"]], [ds[k]["u0"]], [ds[k]["phi"]] if wave[k] else None, out=[us[k]])

    one_by_one()
    ms_1 = timed(one_by_one, 1)
    err_1 = max(mode_error(insts[k], ds[k], us[k]) for k in sample)
    for sv in solvers:
        sv.close()
    mn = sum(i.M * i.N for i in insts)
    for prec in ("fp64", "fp32"):
        ms_b, err_b = batched[prec]
        out["c4_batched_" + prec] = {"ms": round(ms_b, 2), "unknowns_per_s": mn / (ms_b * 1e-3),
                                     "instances": len(insts), "refine_steps": 0 if prec == "fp64" else 1,
                                     "max_error_vs_oracle_sampled": err_b, "sampled_instances": len(sample)}
        log("forms: c4 batched %s %.1f ms (err %.3e)" % (prec, ms_b, err_b))
    out["c4_one_by_one_fp64"] = {"ms": round(ms_1, 2), "unknowns_per_s": mn / (ms_1 * 1e-3),
                                 "max_error_vs_oracle_sampled": err_1}
    out["batched_speedup_vs_fp64"] = round(ms_1 / batched["fp64"][0], 3)
    out["batched_mixed_speedup_vs_fp64"] = round(ms_1 / batched["fp32"][0], 3)
    log("forms: c4 one by one fp64 %.1f ms (err %.3e)" % (ms_1, err_1))
    del ds, us
    torch.cuda.empty_cache()

    # c5: forward solve + adjoint (dL/df, dL/dgamma) of L = ||u - u_obs||^2
    base, obs = wl.c5(build=False)
    db, do = device_inputs(base, dev), device_inputs(obs, dev)
    sv = binding.Solver([dict(gamma=base.gamma, M=base.M, N=base.N)])
    u_obs = sv.solve([do["f"]], [do["u0"]])[0]
    u = torch.empty_like(db["f"])
    fw = lambda: sv.solve([db["f"]], [db["u0"]], out=[u])  # noqa: E731
    fw()
    ms_f = timed(fw, 2)
    g = 2.0 * (u - u_obs)
    lam = torch.empty_like(g)
    holder = {}

    def bw():
        holder["r"] = sv.adjoint([g], [u], [db["u0"]], out=[lam])

    bw()
    ms_a = timed(bw, 2)
    dgamma = float(holder["r"][1][0])
    sv.close()
    # dL/df = lambda: the adjoint of a modal g is modal (modes of base and obs),
    # each the time-reversed scalar recurrence
    import oracle

    _, _, h, _ = wl.grid(base.M, base.N)
    js = sorted(set(db["js"]) | set(do["js"]))
    x, _, _, _ = wl.grid(base.M, base.N)
    S = np.stack([np.sin(j * math.pi * x) for j in js])
    gmodal = (g @ torch.from_numpy(S.T).to(dev)).cpu().numpy() * (2.0 / (base.M + 1))
    lamj = [4.0 / h ** 2 * math.sin(j * math.pi * h / 2) ** 2 for j in js]
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max_workers=len(js)) as ex:
        vs = list(ex.map(lambda k: oracle.mode(base.gamma, base.T, base.N, lamj[k], gmodal[::-1, k].copy(), 0.0,
                                               0.0)[::-1], range(len(js))))
    ref = torch.from_numpy(np.stack(vs, axis=1).copy()).to(dev) @ torch.from_numpy(S).to(dev)
    err_l = float((lam - ref).abs().max() / ref.abs().max())
    out["c5_adjoint"] = {"ms_forward": round(ms_f, 2), "ms_adjoint": round(ms_a, 2), "dL_dgamma": dgamma,
                         "dL_df_error_vs_oracle": err_l}
    log("forms: c5 forward %.1f ms, adjoint %.1f ms, dL/df err %.3e, dL/dgamma %.6e" % (ms_f, ms_a, err_l, dgamma))
    out["gmres_example4"] = run_gmres(dev)
    out["advection"] = run_advection(dev)
    return out


# The paper's timing tables for the advection schemes (h = tau = 2^-k): CPU
# seconds of its fast method on a Matlab PC; context only.
PAPER_ADV_FAST_S = {2: {7: 0.17, 8: 0.43, 9: 1.49, 10: 5.56, 11: 21.4, 12: 399.0},
                    3: {6: 0.14, 7: 0.23, 8: 0.57, 9: 2.01, 10: 6.67, 11: 27.4, 12: 573.0}}


def run_advection(dev, meshes=(6, 7, 8, 9, 10, 11, 12), oracle_upto=11):
    """The advection equations on the paper's timing meshes h = tau = 2^-k:
    Scheme 2 (gamma = 0.9, Example 2 data u = t sin(pi x)) and Scheme 3
    (gamma = 1.5, Example 3 data u = t^3 x (1 - x)).  Time of the recursive
    solve, L2 error at t = T against the exact solution (the paper's
    measure), and the max-norm distance to the oracle's time stepping where
    that finishes in seconds (k <= oracle_upto).  A row whose L2 error at T
    exceeds 1 (the exact solutions are at most 1 in size) is marked
    diverged: Scheme 3 grows without bound from h = tau = 2^-11 on, in the
    oracle's time stepping as much as on the GPU, so those rows time a
    divergent discrete solution."""
    import numpy as np
    import torch

    import oracle
    from paper_1710_11593_amd import binding

    res = {}
    for scheme, gamma in ((2, 0.9), (3, 1.5)):
        rows = {}
        for k in meshes:
            if k not in PAPER_ADV_FAST_S[scheme]:
                continue
            Mp = N = 2 ** k
            M, h = Mp - 1, 1.0 / Mp
            x = h * np.arange(1, Mp)
            if scheme == 2:
                t = np.arange(1, N + 1) / N
                xm = x - h / 2
                f = (np.outer(t ** (1 - gamma) / math.gamma(2 - gamma), np.sin(np.pi * xm))
                     + np.outer(np.pi * t, np.cos(np.pi * xm)))
                exact = np.sin(np.pi * x)
            else:
                th = (np.arange(1, N + 1) - 0.5) / N
                f = (np.outer(6 * th ** (3 - gamma) / math.gamma(4 - gamma), x - x * x)
                     + np.outer(th ** 3, 1 - 2 * x))
                exact = x * (1 - x)
            fd = torch.from_numpy(f).to(dev)
            sv = binding.Solver([dict(gamma=gamma, M=M, N=N)], equation="advection")
            u = torch.empty_like(fd)
            run = lambda: sv.solve([fd], out=[u])  # noqa: E731
            run()
            ms = timed(run, 3)
            sv.close()
            un = u.cpu().numpy()
            row = {"M": M, "N": N, "ms": round(ms, 3), "unknowns_per_s": M * N / (ms * 1e-3),
                   "l2_error_at_T": math.sqrt(h * np.sum((un[-1] - exact) ** 2)),
                   "paper_fast_method_cpu_s": PAPER_ADV_FAST_S[scheme][k]}
            if k <= oracle_upto:
                ref = oracle.solve_adv(gamma, 1.0, 0.0, 1.0, M, N, f)
                row["error_vs_oracle"] = float(np.max(np.abs(un - ref)) / np.max(np.abs(ref)))
                row["oracle_l2_error_at_T"] = math.sqrt(h * np.sum((ref[-1] - exact) ** 2))
            if not row["l2_error_at_T"] <= 1.0:
                row["diverged"] = ("the discrete solution grows without bound (the printed scheme at this mesh; "
                                   + ("the oracle's time stepping diverges the same way)" if k <= oracle_upto
                                      else "not compared with the oracle at this mesh)"))
            rows["h=tau=2^-%d" % k] = row
            log("forms: advection scheme %d gamma %.1f h=tau=2^-%d: %.3f ms, L2 err %.3e%s" % (
                scheme, gamma, k, ms, row["l2_error_at_T"],
                ", vs oracle %.2e" % row["error_vs_oracle"] if "error_vs_oracle" in row else ""))
        res["scheme%d_gamma%.1f" % (scheme, gamma)] = rows
    return res


# The paper's timing table for Scheme 4 (gamma = 0.1, h = tau = 2^-k): CPU
# seconds of its fast (GMRES) method on a Matlab PC; context only.
PAPER_FAST_S = {8: 2.27, 9: 15.6, 10: 263.0}


def run_gmres(dev, meshes=(8, 9, 10), rtol=1e-8):
    """The paper's iterative method, restarted GMRES(m) (section 3.1), on its
    Example 4 data (u = t^3 sin(pi x), gamma = 0.1, h = tau = 2^-k), next to
    the recursive solve of the same system.  Unpreconditioned (the paper's
    method, m = 100) and with the block-diagonal preconditioner (m = 30).
    rtol = 1e-8: at h = 2^-10 the operator's condition number is about 2e6,
    so the relative residual computed in float64 bottoms out near 1e-10 and a
    target there spends most steps restarting on rounding.  Errors against
    the oracle's scalar recurrence of the single sine mode the data carry."""
    import numpy as np
    import torch

    import oracle
    from paper_1710_11593_amd import binding

    gamma = 0.1
    res = {}
    for k in meshes:
        M, N = 2 ** k - 1, 2 ** k
        h = 1.0 / (M + 1)
        x = np.arange(1, M + 1) * h
        t = np.arange(1, N + 1) / N
        G = 6 * t ** (3 - gamma) / math.gamma(4 - gamma) + math.pi ** 2 * t ** 3
        s = np.sin(math.pi * x)
        f = torch.from_numpy(np.outer(G, s)).to(dev)
        lam1 = 4.0 / h ** 2 * math.sin(math.pi * h / 2) ** 2
        ref = torch.from_numpy(np.outer(oracle.mode(gamma, 1.0, N, lam1, G), s)).to(dev)
        sv = binding.Solver([dict(gamma=gamma, M=M, N=N)])
        u = torch.empty_like(f)
        dc = lambda: sv.solve([f], out=[u])  # noqa: E731
        dc()
        ms_dc = timed(dc, 3)
        err_dc = float((u - ref).abs().max() / ref.abs().max())
        row = {"M": M, "N": N, "dc_ms": round(ms_dc, 3), "dc_error_vs_oracle": err_dc,
               "paper_fast_method_cpu_s": PAPER_FAST_S.get(k)}
        for pc, m in ((0, 100), (1, 30)):
            holder = {}

            def run():
                holder["i"] = sv.gmres([f], out=[u], restart=m, max_iters=20000, rtol=rtol, precond=pc)[1][0]

            run()
            ms = timed(run, 1)
            info = holder["i"]
            err = float((u - ref).abs().max() / ref.abs().max())
            key = "gmres" if pc == 0 else "gmres_block_precond"
            row[key] = {"ms": round(ms, 3), "restart": m, "rtol": rtol, "iterations": info["iterations"],
                        "cycles": info["cycles"],
                        "relres": info["relres"], "converged": info["converged"], "error_vs_oracle": err}
            log("forms: gmres h=tau=2^-%d precond %d: %.2f ms, %d steps in %d cycles, err %.2e (recursive solve "
                "%.2f ms)" % (k, pc, ms, info["iterations"], info["cycles"], err, ms_dc))
        sv.close()
        res["h=tau=2^-%d" % k] = row
    return res


PAPER_FCG_S = {9: 0.01, 10: 0.06, 11: 0.09, 12: 0.57, 13: 1.29, 14: 2.24, 15: 4.58, 16: 9.81, 17: 27.2,
               18: 80.9, 19: 281.0, 20: 451.0, 21: 977.0, 22: 2548.0}
PAPER_FCG_ITERS = {9: 62, 10: 75, 11: 91, 12: 110, 13: 133, 14: 159, 15: 192, 16: 230, 17: 276,
                   18: 331, 19: 415, 20: 498, 21: 599, 22: 741}


def run_ode(dev, meshes=tuple(range(9, 23)), gamma=0.5, rtol=1e-10):
    """Scheme 1, the two-sided fractional ODE of Example 1 (u = t(1 - t)),
    by conjugate gradients with the FFT-embedded operator, on the timing
    meshes tau = 2^-9 .. 2^-22 of Table 2.  The table gives neither gamma nor
    the stop rule: gamma = 0.5 reproduces the growth of its step counts
    (about x1.2 per halving of tau, as sqrt(cond) ~ tau^(-gamma/2)), and the
    stop rule here is |r| <= rtol |f|.  Each call includes the set-up of the
    operator (weights and spectra), as the paper's timings include it.  The
    paper's FCG seconds and step counts (Matlab on a desktop) are context."""
    import numpy as np
    import torch

    from paper_1710_11593_amd import binding

    def d(s):
        return s ** (1 - gamma) / math.gamma(2 - gamma) - 2 * s ** (2 - gamma) / math.gamma(3 - gamma)

    res = {}
    for k in meshes:
        N = 2 ** k
        t = np.arange(1, N) / N
        f = torch.from_numpy(d(t) + d(1 - t) + t * (1 - t)).to(dev)
        u = torch.empty_like(f)
        holder = {}

        def run():
            holder["i"] = binding.ode_cg(gamma, N, f, out=u, max_iters=20000, rtol=rtol)[1]

        run()
        ms = timed(run, 3)
        info = holder["i"]
        err = float(np.sqrt(np.sum((u.cpu().numpy() - t * (1 - t)) ** 2) / N))
        res["tau=2^-%d" % k] = {"N": N, "ms": round(ms, 3), "iterations": info["iterations"],
                                "relres": info["relres"], "converged": info["converged"], "l2_error": err,
                                "paper_fcg_cpu_s": PAPER_FCG_S.get(k), "paper_fcg_iterations": PAPER_FCG_ITERS.get(k)}
        log("forms: scheme 1 cg tau=2^-%d: %.2f ms, %d steps, relres %.2e, L2 error %.3e" % (
            k, ms, info["iterations"], info["relres"], err))
    return {"gamma": gamma, "rtol": rtol, "meshes": res}


def run_cpu_full(args):
    """The oracle on the whole configuration, as consecutive row ranges of
    --cpu-block steps (a run split that way computes exactly what one call
    does), each printed when done: the measured full-run time that the
    default cpu_baseline (a bounded sample scaled by (N/steps)^2) estimates."""
    import numpy as np

    import oracle
    from paper_1710_11593_amd import workloads as wl

    inst, desc = build_instance(args)
    M, N, gamma = inst.M, inst.N, inst.gamma
    js, G, c_u0, c_phi = modal_factors(inst)
    x, _, _, _ = wl.grid(M, N)
    S = np.stack([np.sin(j * math.pi * x) for j in js])
    f = np.ascontiguousarray(G @ S)
    u0 = np.asarray(c_u0) @ S
    phi = (np.asarray(c_phi) @ S) if gamma > 1 else None
    u = np.zeros((N, M))
    th = oracle.threads()
    log("cpu-full: %s, oracle on %d threads, blocks of %d steps" % (desc, th, args.cpu_block))
    blocks, t_all = [], 0.0
    for a in range(0, N, args.cpu_block):
        b = min(N, a + args.cpu_block)
        t0 = time.perf_counter()
        oracle.solve_rows(gamma, inst.T, 0.0, 1.0, M, N, f, u, a, b, u0=u0, phi=phi)
        dt = time.perf_counter() - t0
        t_all += dt
        blocks.append({"rows": [a, b], "s": round(dt, 3)})
        log("cpu-full: rows %d..%d in %.2f s (total %.1f s)" % (a, b - 1, dt, t_all))
    sample = sum(bl["s"] for bl in blocks if bl["rows"][1] <= 8192)
    print(json.dumps({"oracle_full_run_s": round(t_all, 2), "threads": th, "M": M, "N": N, "gamma": gamma,
                      "unknowns_per_s": M * N / t_all, "first_8192_steps_s": round(sample, 2),
                      "estimate_from_first_8192_s": round(sample * (N / 8192) ** 2, 1) if N > 8192 else None,
                      "blocks": blocks}),
          flush=True)


def run_batched(args, dev):
    """--config c4: the 256 uneven instances as one batched handle; value =
    sum of M N over the batch per second; error sampled on 8 instances."""
    import torch

    from paper_1710_11593_amd import binding, workloads as wl

    insts = wl.c4()
    ds = [device_inputs(i, dev) for i in insts]
    us = [torch.empty_like(x["f"]) for x in ds]
    wave = [i.gamma > 1 for i in insts]
    prec = args.precision
    ref = args.refine if prec != "fp64" else 0
    sv = binding.Solver([dict(gamma=i.gamma, M=i.M, N=i.N) for i in insts], precision=prec, refine_steps=ref)

    def step():
        sv.solve([x["f"] for x in ds], [x["u0"] for x in ds], [x["phi"] if w else None for x, w in zip(ds, wave)],
                 out=us)

    for _ in range(args.warmup):
        step()
    ms = timed(step, args.steps)
    mn = sum(i.M * i.N for i in insts)
    err = None
    if not args.no_check:
        err = max(mode_error(insts[k], ds[k], us[k]) for k in range(0, len(insts), 32))
    log("bench: c4 batched %s: %.3f ms per solve of 256 instances, error (sampled) %s" % (prec, ms, err))
    sv.set_timing_level(2)
    step()
    torch.cuda.synchronize()
    ks = sv.kernel_stats()
    sv.set_timing_level(0)
    groups = sorted(ks, key=lambda r: -r["ms"])
    for g in groups[:12]:
        log("  %-10s s=%-6d launches=%-6d tasks=%-7d %9.3f ms" % (g["kind"], g["s"], g["launches"], g["tasks"], g["ms"]))
    roof = fft_roofline(ks, prec, 0)
    if roof:
        roof["kernel"] += " (batched, all 256 instances)"
    line = {
        "metric": METRIC, "value": mn / (ms * 1e-3), "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": "c4: 256 uneven instances (M 64..2048, N 2^10..2^15, both regimes), one batched "
                               "handle", "instances": len(insts), "sum_MN": mn, "precision": prec,
                   "refine_steps": ref},
        "error_vs_oracle": err, "roofline": roof, "cpu_baseline": None,
        "kernel_groups": [{"kind": g["kind"], "s": g["s"], "launches": g["launches"], "ms": round(g["ms"], 3)}
                          for g in groups[:10]],
    }
    s = json.dumps(line)
    print(s, flush=True)
    if args.out:
        with open(args.out, "w") as fh_:
            fh_.write(s + "\n")
    sv.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--gamma", type=float, default=0.0)
    ap.add_argument("--M", type=int, default=0)
    ap.add_argument("--N", type=int, default=0)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--refine", type=int, default=1)
    ap.add_argument("--leaf", type=int, default=0)
    ap.add_argument("--crossover", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision (c3), batched (c4) and adjoint (c5) comparisons")
    ap.add_argument("--out", default="")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only time the oracle on the whole configuration (CPU, no GPU), in consecutive "
                         "blocks of --cpu-block time steps, printing each block; the check of the "
                         "cpu_baseline scaling")
    ap.add_argument("--cpu-block", type=int, default=4096)
    ap.add_argument("--solve-once", action="store_true",
                    help="only build the inputs and run one solve of the configuration (the program "
                         "profiled by the HBM counter passes, whose dispatches are then one solve's)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 512 MiB (3 times), the reference kernel for "
                         "scaling HBM counters (FETCH_SIZE / WRITE_SIZE) taken with rocprofv3 --pmc")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        n = (512 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))
        return

    if args.cpu_full:
        return run_cpu_full(args)

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (instances would shard "
              "across GPUs without communication; a single instance does not).  Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    from paper_1710_11593_amd import binding, workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.config == "c4":
        return run_batched(args, dev)
    if args.config == "advection":
        print(json.dumps({"advection": run_advection(dev)}))
        return
    if args.config == "ode":
        # Scheme 1 on Table 2's meshes (with --N 2^k only tau = 2^-k)
        meshes = (int(round(math.log2(args.N))),) if args.N else tuple(range(9, 23))
        print(json.dumps({"scheme1_cg": run_ode(dev, meshes)}))
        return
    if args.config == "gmres":
        # the paper's iterative method on its Example 4 meshes (a form, not the headline)
        meshes = (int(round(math.log2(args.N))),) if args.N else (8, 9, 10)
        print(json.dumps({"gmres_example4": run_gmres(dev, meshes)}))
        return
    inst, desc = build_instance(args)
    M, N, gamma = inst.M, inst.N, inst.gamma
    log("bench: %s, precision %s" % (desc, args.precision))

    # inputs: f = G S with G [N][k] the per-mode time series and S [k][M] the sines
    js, G, c_u0, c_phi = modal_factors(inst)
    x, _, h, tau = wl.grid(M, N)
    S = np.stack([np.sin(j * math.pi * x) for j in js])
    Gd = torch.from_numpy(G).to(dev)
    Sd = torch.from_numpy(S).to(dev)
    f = (Gd @ Sd).contiguous()
    u0 = torch.from_numpy(np.asarray(c_u0) @ S).to(dev)
    phi = torch.from_numpy(np.asarray(c_phi) @ S).to(dev)
    u = torch.empty_like(f)
    torch.cuda.synchronize()

    prec = args.precision
    solver = binding.Solver([dict(gamma=gamma, M=M, N=N)], precision=prec,
                            refine_steps=(args.refine if prec != "fp64" else 0), leaf=args.leaf,
                            crossover=args.crossover)
    wave = gamma > 1.0

    def step():
        solver.solve([f], [u0], [phi] if wave else None, out=[u])

    if args.solve_once:
        step()
        torch.cuda.synchronize()
        log("bench: one solve done")
        return
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = M * N / (ms / 1e3)
    log("bench: %.3f ms per solve, %.4g unknowns/s" % (ms, value))

    # accuracy vs the oracle through single-mode reduction
    err = None
    if not args.no_check:
        from concurrent.futures import ThreadPoolExecutor

        lam = [4.0 / h ** 2 * math.sin(j * math.pi * h / 2) ** 2 for j in js]
        with ThreadPoolExecutor(max_workers=len(js)) as ex:
            vs = list(ex.map(lambda k: oracle.mode(gamma, inst.T, N, lam[k], G[:, k], c_u0[k], c_phi[k]),
                             range(len(js))))
        V = torch.from_numpy(np.stack(vs, axis=1)).to(dev)
        ref = V @ Sd
        err = float((u - ref).abs().max() / ref.abs().max())
        del ref, V
        log("bench: max-norm relative error vs oracle (mode reduction): %.3e" % err)

    # per-kernel timing during one more solve
    solver.set_timing_level(2)
    step()
    torch.cuda.synchronize()
    ks = solver.kernel_stats()
    solver.set_timing_level(0)
    st = solver.stats()
    groups = sorted(ks, key=lambda r: -r["ms"])
    for g in groups[:12]:
        log("  %-10s s=%-6d launches=%-6d %9.3f ms  %8.1f GB/s" % (
            g["kind"], g["s"], g["launches"], g["ms"], g["bytes"] / (g["ms"] * 1e-3) / 1e9 if g["ms"] else 0))
    roof = fft_roofline(ks, prec, M)
    mfma = mfma_levels(ks, M) if prec == "fp64" else []
    leaf = [g for g in ks if g["kind"] == "leaf"]
    leaf_ms = sum(g["ms"] for g in leaf)
    leaf_launches = sum(g["launches"] for g in leaf)
    timed_ms = sum(g["ms"] for g in ks)
    # the sequential chain of leaf solves (one workgroup each) and the level
    # products between them, as shares of the per-group event times
    leaf_s = max((g["s"] for g in groups if g["kind"] == "leaf"), default=st["leaf"])
    critical = {"kernel": "k_leaf_scan (one workgroup per launch, %d time steps of L=%d%s)" % (
                    leaf_s, st["leaf"], ": two leaves and the level product between them" if leaf_s > st["leaf"]
                    else ""),
                "launches": leaf_launches, "avg_us": round(leaf_ms * 1e3 / max(leaf_launches, 1), 2),
                "leaf_share": round(leaf_ms / timed_ms, 3) if timed_ms else None,
                "groups": [{"kind": g["kind"], "s": g["s"], "launches": g["launches"], "ms": round(g["ms"], 3)}
                           for g in groups[:10]]}

    # CPU baseline: the oracle on the first cpu_steps steps at full width
    cpu = None
    if not args.no_cpu_baseline:
        n_s = min(args.cpu_steps, N)
        fh = (G[:n_s] @ S)
        fpad = np.zeros((N, M)) if n_s < N else fh
        if n_s < N:
            fpad[:n_s] = fh
        th = oracle.threads()
        c0 = time.perf_counter()
        oracle.solve(gamma, inst.T, 0.0, 1.0, M, N, fpad, u0=np.asarray(c_u0) @ S,
                     phi=(np.asarray(c_phi) @ S) if wave else None, nsteps=n_s)
        c1 = time.perf_counter()
        rec = recorded_full_run(args.config, M, N, gamma, n_s)
        if rec:
            # the measured ratio of a whole run to this sample on the GPU host
            ratio = rec["total_s"] / rec["first_s"]
            how = ("time scaled by %.2f, the ratio of the whole run (%.1f s on %d threads, measured once, "
                   "profiles/oracle_c2_full_run.md) to its first %d steps" % (ratio, rec["total_s"], rec["threads"],
                                                                             n_s))
        else:
            ratio = (N / n_s) ** 2
            how = "time scaled by (N/%d)^2 to the full run" % n_s
        t_full = (c1 - c0) * ratio
        cpu = {"value": M * N / t_full, "unit": "unknowns/s", "cores": th, "kind": "oracle",
               "sample": "first %d of %d time steps at full M=%d (%.2f s wall); %s" % (n_s, N, M, c1 - c0, how)}
        if rec:
            cpu["full_run_measured_s"] = rec["total_s"]
        log("bench: oracle sample %.2f s on %d threads -> %.4g unknowns/s (full-run estimate)" % (
            c1 - c0, th, cpu["value"]))

    forms = None
    if not args.no_forms and args.config == "c2" and not (args.M or args.N):
        del f, u
        solver.close()
        torch.cuda.empty_cache()
        forms = run_forms(dev)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else ("f32+f64" if prec == "fp32" else "bf16x3+f64"),
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (args.config, desc), "M": M, "N": N, "gamma": gamma,
                   "precision": prec, "leaf": st["leaf"], "crossover": st["crossover"],
                   "refine_steps": args.refine if prec != "fp64" else 0},
        "error_vs_oracle": err,
        "leaf_us_per_step": round(leaf_ms * 1e3 / N, 4) if leaf else None,
        "critical_path": critical,
        "kernels_per_solve": st["kernels"],
        "roofline": roof,
        "mfma": ({"bound": "mfma", "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                  "kernel": "fs::k_dense_mfma (float64 16x16x4 MFMA dense level products)", "levels": mfma}
                 if mfma else None),
        "cpu_baseline": cpu,
        "forms": forms,
    }
    s = json.dumps(line)
    print(s, flush=True)
    if args.out:
        with open(args.out, "w") as fh_:
            fh_.write(s + "\n")
    if forms is None:
        solver.close()


if __name__ == "__main__":
    main()
