#!/usr/bin/env python3
"""Benchmark of the SDMM imaging hot path on one MI355X.

Workload: 1024 x 1024 sky (200 elliptical Gaussians + 2000 point sources),
M = 4194304 continuous visibilities (2-D Gaussian variable-density coverage,
sigma = pi/4), oversampling 2 (2048 x 2048 grid), 8 x 8 Kaiser-Bessel kernel,
SARA (Dirac + Db1..Db8) at 4 levels, input SNR 30 dB.

A step is one SDMM iteration (Algorithm 1): CG x-update with n_cg = 16 on
Q = Phi^dagger Phi + 2I, the l1 prox fused into Psi^dagger, the l2-ball prox
around Phi x, the positivity prox and the next right-hand side, and one
Psi^dagger / Psi pair.  The method counts n_cg + 2 = 18 Phi/Phi^dagger pairs
per iteration; the library applies n_cg + 1 = 17 (the warm-started CG's
initial residual reuses the Phi x of the l2-ball step).  value = visibilities
through the applied pairs per second = M x 17 x steps / time (the rate by the
method's 18 is reported beside it).  Inputs are resident in HBM before the
timed region.  FP32 storage and arithmetic with FP64 norms and CG scalars.

The SDMM iterations are timed twice on the same plan and data: enqueued as
stream launches (riop_sdmm), and as a one-channel batch whose iterations are
one captured HIP graph replayed (riop_batch_sdmm); the faster is `value` and
`config.launch` says which.  Neither timed region records timing events;
per-kernel times and the roofline of the dominant kernel come from a separate
short run with HIP events on the library's stream.

Also reported: SDMM iterations/s, the same in plain FP64, stand-alone
Phi + Phi^dagger pair throughput, a measured device-copy ceiling beside the
8 TB/s peak, the FP32 path's errors against FP64 (this workload) and against
the oracle (64^2), the 64^2 and 256^2 throughputs, Q applied through the
stored G^T G against degridding + gridding, and the CPU oracle on a bounded
pair (one core and all cores, per pair and per SDMM iteration).
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

METRIC = "visibilities/s through Phi+Phi^dagger and SDMM iters/s at 1024^2, FP32 vs FP64 plain"
HBM_PEAK_GBS = 8000.0
GRID_SOURCE = os.path.join(ROOT, "paper_1307_4370_amd", "csrc", "gridding.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "grid_fp32_1024sq_M4194304_hbm_traffic.md")


def source_hash(path=GRID_SOURCE):
    import hashlib
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per FP32 gridding launch from the committed counter summary, or None
    when the summary is missing or was taken on a different gridding source."""
    import re
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    h = re.search(r"gridding source sha256/16: `([0-9a-f]+)`", text)
    b = re.search(r"HBM bytes per gridding launch: `([0-9.e+]+)`", text)
    if not h or not b or h.group(1) != source_hash():
        return None
    return float(b.group(1))


def traffic_summary(fetch_dir, write_dir, probe_mib):
    """Write the HBM-traffic summary of the FP32 gridding launch from two rocprofv3
    --pmc runs (FETCH_SIZE, then WRITE_SIZE), each calibrated on a plain device copy
    of probe_mib MiB (the largest __amd_rocclr_copyBuffer dispatch of the run)."""
    import csv, glob, collections

    def per_dispatch(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        vals = collections.defaultdict(float)
        names = {}
        for f in files:
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                key = (f, r["Dispatch_Id"])
                vals[key] += float(r["Counter_Value"])
                names[key] = r["Kernel_Name"]
        return [(names[k], v * 1024.0) for k, v in vals.items()]  # KiB -> bytes

    probe = probe_mib * 2 ** 20
    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = per_dispatch(d, counter)
        copies = [v for n, v in rows if "copyBuffer" in n]
        cal = probe / max(copies) if copies else 1.0
        tile = [v for n, v in rows if "grid_tile<float, 8, false" in n and ", true>(" not in n]
        merge = [v for n, v in rows if "grid_merge<float>" in n]
        t = sum(tile) / len(tile) if tile else 0.0
        m = sum(merge) / len(merge) if merge else 0.0
        out[counter] = dict(cal=cal, tile=t * cal, merge=m * cal, n_tile=len(tile), n_merge=len(merge),
                            probe_raw=max(copies) if copies else 0.0)
    total = sum(out[c]["tile"] + out[c]["merge"] for c in out)
    lines = ["# HBM traffic of the FP32 gridding launch, 1024^2, M = 4194304, J = 8 (grid_tile; grid_merge only where the "
             "adjoint FFT does not add the halos itself)\n",
             "Commands (repository root on the MI355X host, one counter pass each; $OUT is any writable folder):\n", "```",
             "cd /tmp && export TMPDIR=/tmp",
             f"timeout -s KILL 150 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/pmc_fetch -o t -- "
             f"python3 $REPO/bench.py --steps 1 --warmup 1 --pairs 2 --no-cpu-baseline --no-fp64 --no-graph --no-batch --no-extras --copy-probe {probe_mib}",
             f"timeout -s KILL 150 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/pmc_write -o t -- "
             f"python3 $REPO/bench.py --steps 1 --warmup 1 --pairs 2 --no-cpu-baseline --no-fp64 --no-graph --no-batch --no-extras --copy-probe {probe_mib}",
             f"python3 $REPO/bench.py --traffic-summary $OUT/pmc_fetch $OUT/pmc_write "
             f"--copy-probe {probe_mib}", "```\n",
             f"Calibration: a plain {probe_mib} MiB device copy; its counter reading is scaled to exactly "
             f"{probe_mib} MiB read and written.\n",
             "| counter | copy-probe reading (bytes) | factor | grid_tile per launch (bytes) | grid_merge per launch (bytes) | launches |",
             "|---|---:|---:|---:|---:|---:|"]
    for c in out:
        o = out[c]
        lines.append(f"| {c} | {o['probe_raw']:.4g} | {o['cal']:.4f} | {o['tile']:.4g} | {o['merge']:.4g} | "
                     f"{o['n_tile']}/{o['n_merge']} |")
    lines += ["", f"HBM bytes per gridding launch: `{total:.6g}`", "",
              f"Algorithmic bytes per launch (32N + 16M, FP32): {algorithmic_bytes('grid', 1024, 4194304, 8):.6g}", "",
              f"gridding source sha256/16: `{source_hash()}`", ""]
    open(TRAFFIC_FILE, "w").write("\n".join(lines))
    print("\n".join(lines))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(kind: str, n: int, M: int, cbytes: int, J: int = 8):
    """Bytes the method must move per launch of one kernel kind.

    N = n^2 pixels, grid K^2 = 4N cells; complex = cbytes, (u, v) = cbytes.
      fft_fwd_col: read x (N), write the K x n intermediate (2N)      -> 3N complex
      fft_fwd_row: read 2N, write the grid 4N                         -> 6N
      fft_adj_row: read the grid 4N, write 2N                         -> 6N
      fft_adj_col: read 2N, write x N                                 -> 3N
      degrid:      read the grid 4N + (u, v) M, write y M            -> 4N + 2M
      grid:        read (u, v) M + values M, write the grid 4N       -> 4N + 2M
      grid_zero:   write the grid 4N
      gram:        read the J + (J-1)(2J-1) real planes of G^T G (half a
                   complex each per cell), read the grid 4N, write 4N
    """
    N = n * n
    planes = J + (J - 1) * (2 * J - 1)
    table = {"gram": 4 * N * 2 + 4 * N * planes / 2, "fft_fwd_col": 3 * N, "fft_fwd_row": 6 * N, "fft_adj_row": 6 * N, "fft_adj_col": 3 * N,
             "degrid": 4 * N + 2 * M, "grid": 4 * N + 2 * M, "grid_zero": 4 * N}
    return table[kind] * cbytes if kind in table else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_pair_time(args):
    """One oracle Phi + Phi^dagger pair on the given visibilities, best of
    `pairs`: (seconds in the full-size grid FFTs, seconds in the interpolation
    G then G^T).  Building G is not timed."""
    n, J, uv, x, pairs = args
    import numpy as np
    from oracle import nufft
    op = nufft.Operator(n, uv, J)
    t_fft = t_int = math.inf
    for _ in range(pairs):
        t0 = time.perf_counter()
        X = op.forward_grid(x)
        t1 = time.perf_counter()
        grid = op.grid_adj(op.degrid(X))
        t2 = time.perf_counter()
        np.fft.ifft2(grid)
        t3 = time.perf_counter()
        t_fft = min(t_fft, (t1 - t0) + (t3 - t2))
        t_int = min(t_int, t2 - t1)
    return t_fft, t_int


def cpu_baseline(n, J, L, uv, x_true, ncg, share=4, pairs=2):
    """The FP64 oracle on the host, per Phi/Phi^dagger pair and per SDMM
    iteration of the 1024^2 workload, from a bounded sample.

    One core (the oracle as it is: numpy's FFT and scipy's sparse products run
    on one thread): a pair with the full-size 2048^2 FFTs and the
    interpolation (G, G^T) on the first M / `share` visibilities, the
    interpolation time scaled by `share` (its cost is linear in M apart from
    G^T's grid-sized part, a few per cent that the scaling counts `share`
    times); and one Psi^dagger / Psi pair of the 9-basis dictionary.  An SDMM
    iteration is taken as (n_cg + 2) pairs, as the method counts them, plus the
    Psi pair (the prox and vector steps are small against these).  All cores
    (capped at 16): the M visibilities split into one share per core, one
    oracle process per share, all timed together, each with the full-size
    FFTs; the pair time is the slowest share's, unscaled (summing the shares'
    grids is not counted).
    """
    import numpy as np
    from oracle import wavelets
    M = len(uv)
    m = M // share
    x = x_true.astype(np.complex128)
    t_fft, t_int = _oracle_pair_time((n, J, uv[:m], x, pairs))
    per_pair_1 = t_fft + t_int * (M / m)
    sara = wavelets.Sara(n, L)
    t0 = time.perf_counter()
    sara.psi(sara.psi_adj(x))
    t_psi = time.perf_counter() - t0
    per_iter_1 = (ncg + 2) * per_pair_1 + t_psi
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = min(avail, 16)
    all_cores = None
    if cores > 1:
        import concurrent.futures as cf
        import multiprocessing as mp
        shares = np.array_split(uv, cores)
        with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
            per = max(tf + ti for tf, ti in ex.map(_oracle_pair_time, [(n, J, sh, x, 1) for sh in shares]))
        all_cores = {"cores": cores, "visibilities_per_s": M / per, "seconds_per_pair": per,
                     "sdmm_iters_per_s": 1.0 / ((ncg + 2) * per + t_psi),
                     "note": "the M visibilities split over one oracle process per core, each with the "
                             "full-size FFTs; grid sum and Psi pair not split"}
    return {
        "value": M / per_pair_1, "unit": "visibilities/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 oracle pair on the 1024^2 workload: full-size 2048^2 FFTs, interpolation on "
                   f"{m} of {M} visibilities scaled by {M / m:g} (G build not timed), best of {pairs}; "
                   f"plus one 9-basis Psi pair; SDMM iteration = {ncg + 2} pairs + the Psi pair"),
        "seconds_per_pair": per_pair_1,
        "seconds_fft_per_pair": t_fft,
        "seconds_psi_pair": t_psi,
        "seconds_per_sdmm_iteration": per_iter_1,
        "sdmm_iters_per_s": 1.0 / per_iter_1,
        "all_cores": all_cores,
        "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(), "cpus_available": avail,
    }


def copy_ceiling(dev, mib=1024, reps=10):
    """Device-to-device copy bandwidth (read + write bytes / time)."""
    import torch
    nb = mib * 2 ** 20
    src = torch.empty(nb, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - a) / reps
    del src, dst
    return 2 * nb / dt / 1e9


def small_workloads(dev, steps=20):
    """Throughput of the 64^2 (M = 2048, J = 6) and 256^2 (M = 131072, J = 8)
    workloads: SDMM iterations/s with n_cg = 16 and Phi + Phi^dagger pairs/s,
    FP32 and FP64, as stream launches (inputs resident)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1307_4370_amd import Plan
    out = {}
    for c in (W.C1, W.C2):
        x_true, uv = W.config_inputs(c)
        row = {}
        for prec in ("f32", "f64"):
            rd = torch.float32 if prec == "f32" else torch.float64
            cd = torch.complex64 if prec == "f32" else torch.complex128
            plan = Plan(c.n, torch.tensor(uv, device=dev).to(rd), J=c.J, levels=c.levels, prec=prec)
            xd = torch.tensor(x_true, device=dev).to(cd)
            y = plan.phi(xd)
            eps = 0.05 * float(torch.linalg.vector_norm(y))
            plan.sdmm(y, eps, T=2, n_cg=c.n_cg)
            torch.cuda.synchronize()
            a = time.perf_counter()
            plan.sdmm(y, eps, T=steps, n_cg=c.n_cg)
            torch.cuda.synchronize()
            it_s = steps / (time.perf_counter() - a)
            for _ in range(3):
                plan.phi_adj(plan.phi(xd, y, sorted=True), sorted=True)
            torch.cuda.synchronize()
            a = time.perf_counter()
            for _ in range(50):
                plan.phi_adj(plan.phi(xd, y, sorted=True), sorted=True)
            torch.cuda.synchronize()
            pair_s = 50 / (time.perf_counter() - a)
            row[prec] = {"sdmm_iters_per_s": round(it_s, 2), "pairs_per_s": round(pair_s, 1),
                         "visibilities_per_s": c.M * pair_s}
            del plan
        out[c.name] = {"n": c.n, "M": c.M, "J": c.J, **row}
    log(f"small workloads: {out}")
    return out


def gram_crossover(dev):
    """Q = Phi^dagger Phi + 2I with the stored G^T G against degridding and
    gridding, FP32, J = 8: where M >> K^2 (256^2, M = 8388608) and at the
    benchmark's M = K^2 (1024^2, M = 4194304)."""
    import torch

    import workloads as W
    from paper_1307_4370_amd import Plan
    rows = []
    for n, M in ((256, 8388608), (1024, 4194304)):
        uv = W.coverage(M, W.rng(700, n))
        plan = Plan(n, torch.tensor(uv, device=dev).float(), J=8, levels=1, dict_mask=1, prec="f32")
        x = torch.ones(n, n, dtype=torch.complex64, device=dev)

        def q_us(reps=10):
            for _ in range(3):
                plan.apply_q(x)
            torch.cuda.synchronize()
            a = time.perf_counter()
            for _ in range(reps):
                plan.apply_q(x)
            torch.cuda.synchronize()
            return (time.perf_counter() - a) * 1e6 / reps

        plain = q_us()
        a = time.perf_counter()
        plan.gram_build()
        torch.cuda.synchronize()
        build = time.perf_counter() - a
        gram = q_us()
        rows.append({"n": n, "M": M, "K2": (2 * n) ** 2, "us_per_Q_degrid_grid": round(plain, 1),
                     "us_per_Q_stored_gram": round(gram, 1), "build_s": round(build, 3),
                     "plan_device_GB": round(plan.info()["device_bytes"] / 1e9, 3)})
        del plan
        torch.cuda.empty_cache()
    log(f"gram crossover: {rows}")
    return rows


def s1_errors(xa, sta, ha, xb, stb, hb, T):
    """Relative errors of result a against reference b: the iterate (L2), nu,
    gamma and f1 after the last iteration."""
    import torch
    xr = float(torch.linalg.vector_norm(xa.to(xb.dtype) - xb) / torch.linalg.vector_norm(xb))

    def r(a, b):
        return abs(a - b) / abs(b) if b else abs(a - b)
    return {"iterations": T, "xhat_rel_l2": xr, "nu_rel": r(sta["nu"], stb["nu"]),
            "gamma_rel": r(sta["gamma"], stb["gamma"]), "f1_rel": r(ha[-1][0], hb[-1][0])}


def s1_vs_oracle(dev, T=20):
    """The FP32 GPU path against the FP64 oracle on the 64^2 workload (M = 2048,
    J = 6, 3 levels, n_cg = 16), T iterations from zero, both on the FP32-rounded
    (u, v) and y so that only the arithmetic differs."""
    import numpy as np
    import torch

    import workloads as W
    from oracle import nufft, sdmm as osdmm, wavelets
    from paper_1307_4370_amd import Plan
    c = W.C1
    x_true, uv = W.config_inputs(c)
    uv = uv.astype(np.float32).astype(np.float64)
    op = nufft.Operator(c.n, uv, c.J)
    y0 = op.phi(x_true)
    sig = osdmm.noise_sigma(y0, c.isnr_db)
    y = (y0 + sig * W.unit_complex_noise(c.M, W.rng(c.cfg, W.STREAM_NOISE))).astype(np.complex64)
    eps = osdmm.noise_bound(c.M, sig)
    xo, _, hist, gam = osdmm.sdmm(y.astype(np.complex128), eps, op, wavelets.Sara(c.n, c.levels), T, c.n_cg)
    plan = Plan(c.n, torch.tensor(uv, device=dev).float(), J=c.J, levels=c.levels, prec="f32")
    xg, st, gh, _ = plan.sdmm(torch.tensor(y, device=dev), eps, T=T, n_cg=c.n_cg)
    torch.cuda.synchronize()
    ref_st = {"nu": hist[-1]["nu"], "gamma": gam}
    out = s1_errors(xg, st, gh, torch.tensor(xo, device=dev), ref_st, [[hist[-1]["f1"]]], T)
    del plan
    return out


def batch_vs_plain(steps, ncg, dev):
    """System form S2 against the plain form on the uneven multi-channel workload.

    32 channels (image sides 128..512, M = 1..4 N per channel, frequency
    scale 1..2), FP32, J = 8, SARA at 4 levels: the same `steps` SDMM
    iterations (from x = 0, each channel's gamma set up as in Algorithm 1's
    initialisation) once as one batch (one
    replayed HIP graph over all channels, tiles from the autotuner) and once
    as a loop of per-channel riop_sdmm calls (stream launches, each call
    ending in a host wait), and a third time with every channel's set-up and
    iterations enqueued on one stream without host waits (riop_sdmm_init /
    riop_sdmm_step) and collected at the end.  Reports visibilities/s through
    Phi+Phi^dagger for all three and the largest relative differences between
    the forms' iterates.  y = Phi x + noise at 30 dB
    ISNR with this library's Phi (throughput input only).
    """
    import numpy as np
    import torch

    import workloads as W
    from paper_1307_4370_amd import Batch, Plan, noise_bound

    cfg, J, L = 4, 8, 4
    chans = W.batch_channels(32, cfg)
    plans, uvs, ys, eps = [], [], [], []
    for k, (n, M, f) in enumerate(chans):
        g = W.rng(cfg, W.STREAM_UV, k)
        uv = torch.tensor(W.coverage(M, g, scale=f).astype(np.float32), device=dev)
        sc = (n / 256) ** 2
        x = W.sky(n, max(1, round(80 * sc)), max(1, round(400 * sc)), W.rng(cfg, W.STREAM_SKY, k))
        plan = Plan(n, uv, J=J, levels=L, prec="f32")
        y0 = plan.phi(torch.tensor(x, device=dev).to(torch.complex64)).cpu().numpy().astype(np.complex128)
        sigma = float(np.linalg.norm(y0)) * 10 ** (-30.0 / 20) / math.sqrt(M)
        y = y0 + sigma * W.unit_complex_noise(M, W.rng(cfg, W.STREAM_NOISE, k))
        plans.append(plan)
        uvs.append(uv)
        ys.append(torch.tensor(y, device=dev).to(torch.complex64))
        eps.append(noise_bound(M, sigma))
    Ms = [M for _, M, _ in chans]
    t0 = time.perf_counter()
    bt = Batch([(n, uv) for (n, _, _), uv in zip(chans, uvs)], J=J, levels=L, prec="f32", autotune=True)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0

    def run_plain():
        return [plan.sdmm(y, e, T=steps, n_cg=ncg)[0] for plan, y, e in zip(plans, ys, eps)]

    run_plain()
    torch.cuda.synchronize()
    a = time.perf_counter()
    xp = run_plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - a
    # The same iterations enqueued for all channels on one stream with no
    # host wait between channels (riop_sdmm_init / riop_sdmm_step), collected
    # at the end: the plain form without its per-channel synchronisation.
    def run_enqueued():
        for plan, y, e in zip(plans, ys, eps):
            plan.sdmm_enqueue(y, e, T=steps, n_cg=ncg)
        return [plan.sdmm_collect()[0] for plan in plans]

    run_enqueued()
    torch.cuda.synchronize()
    a = time.perf_counter()
    xq = run_enqueued()
    torch.cuda.synchronize()
    t_enq = time.perf_counter() - a
    bt.sdmm(ys, eps, T=steps, n_cg=ncg, iters_per_graph=steps)
    torch.cuda.synchronize()
    a = time.perf_counter()
    xb, stb = bt.sdmm(ys, eps, T=steps, n_cg=ncg, iters_per_graph=steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - a
    diff = max(float(torch.linalg.vector_norm(b - q) / max(float(torch.linalg.vector_norm(q)), 1e-300))
               for b, q in zip(xb, xp))
    diff_q = max(float(torch.linalg.vector_norm(b - q) / max(float(torch.linalg.vector_norm(q)), 1e-300))
                 for b, q in zip(xq, xp))
    pairs = sum(Ms) * (ncg + 1) * steps
    out = {"channels": len(chans), "visibilities": sum(Ms), "sides": sorted({n for n, _, _ in chans}),
           "steps": steps, "n_cg": ncg,
           "batch_visibilities_per_s": pairs / t_batch, "plain_visibilities_per_s": pairs / t_plain,
           "speedup": t_plain / t_batch, "max_rel_diff_batch_vs_plain": diff,
           "enqueued_visibilities_per_s": pairs / t_enq, "speedup_vs_enqueued": t_enq / t_batch,
           "max_rel_diff_enqueued_vs_plain": diff_q,
           "batch_setup_s": round(t_setup, 3),
           "note": "both forms run the same steps from x = 0, including each channel's gamma set-up"}
    log(f"batch S2: {out}")
    bt.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-cg", type=int, default=16)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--pairs", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched (S2) vs per-channel comparison")
    ap.add_argument("--batch-steps", type=int, default=4)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the copy ceiling, the 64^2 / 256^2 throughputs and the Gram comparison")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="after the run, copy this many MiB device to device (counter calibration)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the gridding HBM-traffic summary from two rocprofv3 --pmc output folders and exit")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(args.traffic_summary[0], args.traffic_summary[1], args.copy_probe or 512)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(sharding the visibilities across GPUs is not implemented); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_1307_4370_amd import Batch, Plan, noise_bound

    c = W.C3
    n, M, J, L, ncg = c.n, c.M, c.J, c.levels, args.n_cg
    dev = torch.device("cuda:0")
    log(f"workload n={n} M={M} J={J} levels={L} n_cg={ncg}")
    x_true, uv = W.config_inputs(c)
    noise = W.unit_complex_noise(M, W.rng(c.cfg, W.STREAM_NOISE))

    def setup(prec):
        rd = np.float32 if prec == "f32" else np.float64
        cd = torch.complex64 if prec == "f32" else torch.complex128
        uvd = torch.tensor(uv.astype(rd), device=dev)
        plan = Plan(n, uvd, J=J, levels=L, prec=prec)
        xd = torch.tensor(x_true, device=dev).to(cd)
        y0 = plan.phi(xd)
        torch.cuda.synchronize()
        y0h = y0.cpu().numpy().astype(np.complex128)
        sigma = float(np.linalg.norm(y0h)) * 10 ** (-c.isnr_db / 20) / math.sqrt(M)
        y = torch.tensor(y0h + sigma * noise, device=dev).to(cd)
        eps = noise_bound(M, sigma)
        return plan, xd, y, eps

    # ---- FP32 SDMM (the timed steps) -----------------------------------------
    plan, xd, y, eps = setup("f32")
    log(f"plan: {plan.info()}")
    x, st, _, state = plan.sdmm(y, eps, T=args.warmup, n_cg=ncg)
    gamma = st["gamma"]
    torch.cuda.synchronize()
    # (1) stream launches, no timing events in the timed region.
    t0 = time.perf_counter()
    x, st, hist, state = plan.sdmm(y, eps, T=args.steps, n_cg=ncg, gamma=gamma, x0=x, state=state)
    torch.cuda.synchronize()
    ms_stream = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"fp32 stream launches: {ms_stream:.3f} ms/iteration, nu={st['nu']:.4f}")
    # (2) per-kernel times from HIP events on the library stream (separate run).
    ev_steps = max(1, min(args.steps, 3))
    plan.timing(True)
    torch.cuda.synchronize()
    plan.sdmm(y, eps, T=ev_steps, n_cg=ncg, gamma=gamma, x0=x, state=state)
    torch.cuda.synchronize()
    kernels = plan.timing_read()
    plan.timing(False)
    # (3) the same solve as a one-channel batch: one captured HIP graph of
    # `steps` iterations, replayed; iteration time = (t(2 steps) - t(steps)) / steps.
    ms_graph = None
    if not args.no_graph:
        bt = Batch([(n, plan._uv)], J=J, levels=L, prec="f32", autotune=False)
        bt.sdmm([y], [eps], T=args.steps, n_cg=ncg, gamma=gamma, iters_per_graph=args.steps)
        torch.cuda.synchronize()
        a = time.perf_counter()
        bt.sdmm([y], [eps], T=args.steps, n_cg=ncg, gamma=gamma, iters_per_graph=args.steps)
        torch.cuda.synchronize()
        b = time.perf_counter()
        bt.sdmm([y], [eps], T=2 * args.steps, n_cg=ncg, gamma=gamma, iters_per_graph=args.steps)
        torch.cuda.synchronize()
        c2 = time.perf_counter()
        ms_graph = ((c2 - b) - (b - a)) * 1e3 / args.steps
        log(f"fp32 graph replay: {ms_graph:.3f} ms/iteration")
        bt.close()
        del bt
    ms_step = min(ms_stream, ms_graph) if ms_graph else ms_stream
    launch = "hip graph replay" if ms_graph and ms_graph <= ms_stream else "stream launches"
    # The method's count is n_cg + 2 pairs per iteration (n_cg + 1 in CG with a
    # warm start, one in steps 7-9); the library applies n_cg + 1 of each
    # operator (the warm start's Phi^dagger Phi xhat is folded into the carried
    # right-hand side), and `value` counts the pairs it applies.
    pairs_per_step = ncg + 1
    method_pairs_per_step = ncg + 2
    value = M * pairs_per_step / (ms_step * 1e-3)
    iters_s = 1e3 / ms_step
    log(f"fp32: {ms_step:.3f} ms/iteration ({launch}), {value:.4g} vis/s")

    # Roofline of the dominant kernel (largest total time in the timed region).
    cb = 8
    dom = max((k for k in kernels if algorithmic_bytes(k, n, M, cb) is not None), key=lambda k: kernels[k][0])
    tot_ms, launches = kernels[dom]
    avg_s = tot_ms * 1e-3 / max(1, launches)
    ach = algorithmic_bytes(dom, n, M, cb) / avg_s / 1e9
    traffic = recorded_traffic() if dom == "grid" else None
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "avg_launch_us": round(avg_s * 1e6, 2)}
    kern = {k: {"total_ms": round(v[0], 3), "launches": v[1],
                "avg_us": round(v[0] * 1e3 / v[1], 2) if v[1] else None,
                "algorithmic_GBs": (round(algorithmic_bytes(k, n, M, cb) / (v[0] * 1e-3 / v[1]) / 1e9, 1)
                                    if v[1] and algorithmic_bytes(k, n, M, cb) else None)}
            for k, v in kernels.items() if v[1]}

    # A whole solve of this workload from x = 0: its T iterations (Algorithm 1
    # with the same parameters), timed, and the reconstruction quality of the
    # synthetic sky (SNR = 20 log10 ||x|| / ||x - Re x_hat||).
    solve = None
    if not args.no_extras:
        torch.cuda.synchronize()
        a = time.perf_counter()
        xs, sts, _, _ = plan.sdmm(y, eps, T=c.T, n_cg=ncg)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - a
        xr = xs.real.double().cpu().numpy()
        snr = 20 * math.log10(float(np.linalg.norm(x_true)) / float(np.linalg.norm(x_true - xr)))
        solve = {"iterations": sts["iters"], "seconds": round(t_solve, 3), "nu": sts["nu"], "zeta": sts["zeta"],
                 "snr_db": round(snr, 2), "note": "FP32, from x = 0, stream launches; set-up included"}
        log(f"solve: {solve}")

    # Stand-alone Phi + Phi^dagger pairs (caller order and plan order).
    def pair_rate(p, xin, yin, sorted_, reps):
        for _ in range(2):
            p.phi_adj(p.phi(xin, yin, sorted=sorted_), sorted=sorted_)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            p.phi_adj(p.phi(xin, yin, sorted=sorted_), sorted=sorted_)
        torch.cuda.synchronize()
        return M * reps / (time.perf_counter() - a)

    ybuf = torch.empty(M, dtype=torch.complex64, device=dev)
    pairs32 = {"caller_order": pair_rate(plan, xd, ybuf, False, args.pairs),
               "plan_order": pair_rate(plan, xd, ybuf, True, args.pairs)}
    log(f"fp32 pairs: {pairs32}")
    del ybuf

    fp64 = None
    s1 = {}
    if not args.no_fp64:
        plan64, xd64, y64, eps64 = setup("f64")
        x64, st64, _, state64 = plan64.sdmm(y64, eps64, T=1, n_cg=ncg)
        torch.cuda.synchronize()
        a = time.perf_counter()
        x64, st64, h64, state64 = plan64.sdmm(y64, eps64, T=args.fp64_steps, n_cg=ncg, gamma=st64["gamma"],
                                              x0=x64, state=state64)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - a) * 1e3 / args.fp64_steps
        yb64 = torch.empty(M, dtype=torch.complex128, device=dev)
        fp64 = {"ms_per_step": round(ms64, 3), "sdmm_iters_per_s": round(1e3 / ms64, 3),
                "visibilities_per_s": M * pairs_per_step / (ms64 * 1e-3),
                "pair_visibilities_per_s": pair_rate(plan64, xd64, yb64, False, max(2, args.pairs // 4))}
        log(f"fp64: {fp64}")
        # FP32 against FP64 on this workload: the same measured data (the FP64
        # y rounded to FP32), each path from zero for 1 + fp64_steps iterations
        # with its own gamma.
        T1 = 1 + args.fp64_steps
        x32, st32, h32, _ = plan.sdmm(y64.to(torch.complex64), eps64, T=T1, n_cg=ncg)
        torch.cuda.synchronize()
        s1["fp32_vs_fp64_1024"] = s1_errors(x32, st32, h32, x64, st64, h64, T1)
        log(f"S1 1024^2: {s1['fp32_vs_fp64_1024']}")
        del plan64, yb64, x32

    if args.copy_probe:
        nb = args.copy_probe * 2 ** 20
        src = torch.empty(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe} MiB x 3")
        del src, dst

    extras = {}
    if not args.no_extras:
        extras["copy_GBs"] = copy_ceiling(dev)
        log(f"device copy: {extras['copy_GBs']:.1f} GB/s")
        extras["small"] = small_workloads(dev)
        extras["gram"] = gram_crossover(dev)
    if "copy_GBs" in extras:
        roofline["copy_ceiling_GBs"] = round(extras["copy_GBs"], 1)
        roofline["frac_of_copy"] = round(ach / extras["copy_GBs"], 4)

    s2 = None
    if not args.no_batch:
        s2 = batch_vs_plain(args.batch_steps, ncg, dev)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(n, J, L, uv, x_true, ncg)
        log(f"cpu: {cpu}")
        s1["fp32_vs_oracle_64"] = s1_vs_oracle(dev)
        log(f"S1 64^2: {s1['fp32_vs_oracle_64']}")

    out = {
        "metric": METRIC, "value": value, "unit": "visibilities/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"{c.name}: {n}x{n} sky, M={M} Gaussian-density (u,v), oversampling 2, "
                                f"KB J={J}, SARA Dirac+Db1-8 at {L} levels, one SDMM iteration per step "
                                f"with n_cg={ncg}"),
                   "n": n, "M": M, "J": J, "levels": L, "n_cg": ncg, "pairs_per_step": pairs_per_step,
                   "method_pairs_per_step": method_pairs_per_step,
                   "launch": launch},
        "sdmm_iters_per_s": round(iters_s, 3),
        "method_visibilities_per_s": M * method_pairs_per_step / (ms_step * 1e-3),
        "ms_per_step_stream": round(ms_stream, 4),
        "ms_per_step_graph": round(ms_graph, 4) if ms_graph else None,
        "pair_visibilities_per_s": pairs32,
        "fp64": fp64,
        "roofline": roofline,
        "kernels": kern,
        "cpu_baseline": cpu,
        "s1_errors": s1 or None,
        "solve": solve,
        "small_workloads": extras.get("small"),
        "gram_vs_degrid_grid": extras.get("gram"),
        "batch_s2": s2,
        "final_nu": st["nu"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
