#!/usr/bin/env python3
"""Stationary-PDF throughput on one MI355X.

Workload (default): a 64x64 pixel array, N=1024 bins over a 100 ns period,
dead time 50 ns, pulse sigma 0.4 ns, depth U[5,95] ns, signal flux
log-uniform [0.05,5], background log-uniform [0.01,1] (seed 3); float32
build and sweeps with a float64 residual check; every pixel solved to
L1 <= 1e-6.  One step = one dtm_solve_batched call over all pixels: bin
tables, shifted transition matrices, power iteration, float64 check.  Inputs
(scene metadata) are resident in HBM before the timed region.

Prints one JSON line.  --gpus above 1 is refused: the solver runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor peak
KERNEL_SOURCES = ("dtm_kernels.hip", "dtm_device.hpp", "dtm_internal.h", "dtm_host.cpp")


def kernel_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_20500_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/*.md, line 'traffic-record: ...'), or None when there is none
    for this kernel and workload or the kernel sources changed since."""
    import glob
    sha = kernel_sources_sha1()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("sha1") == sha:
                    return float(kv["bytes"])
    return None


MC_SOURCES = ("dtm_mc.hip", "dtm_internal.h", "dtm_host.cpp")
FACT_SOURCES = ("dtm_factored.hip", "dtm_device.hpp", "dtm_internal.h", "dtm_host.cpp")
VALU_PEAK_G = 256 * 4 * 2.4e9 / 4 / 1e9  # wave64 VALU instructions/s: 256 CUs x 4 SIMDs, 4 cycles each


def sources_sha1(files):
    import hashlib
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, "paper_2509_20500_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_record(tag, kernel, workload, files):
    """Value of a 'tag: kernel=... workload=... sha1=... value=...' line in
    the committed rocprofv3 summaries (profiles/*.md), or None when there is
    none for these sources."""
    import glob
    sha = sources_sha1(files)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith(tag + ":"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("sha1") == sha:
                    return float(kv["value"])
    return None


def progress(msg):
    """A phase line on stderr (the JSON result alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def _mc_oracle_one(rec):
    import numpy as np

    from oracle import mc_philox
    fields, cycles, seed, run, pixel = rec
    h = np.zeros(fields[6], dtype=np.int64)
    mc_philox.simulate_run(fields, cycles, 0, seed, run, pixel, h)
    return int(h.sum())


def mc_cpu_baseline(scenes, cycles=6000, runs=4):
    """The counter-based oracle simulator (pure Python) on a bounded sample:
    `runs` runs of `cycles` periods for every scene, one process per host
    core (capped at 16)."""
    import multiprocessing as mp
    workers = max(1, min(os.cpu_count() or 1, 16))
    recs = []
    for p, s in enumerate(scenes):
        f = (float(s["period_ns"]), float(s["dead_time_ns"]), float(s["pulse_center_ns"]),
             float(s["pulse_sigma_ns"]), float(s["signal_flux"]), float(s["background_flux"]),
             int(s["n_bins"]))
        recs += [(f, cycles, 5, r, p) for r in range(runs)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_noop, range(workers))
        t0 = time.perf_counter()
        pool.map(_mc_oracle_one, recs, chunksize=1)
        dt = time.perf_counter() - t0
    periods = len(recs) * cycles
    return {"value": periods / dt, "unit": "laser periods/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(scenes)} scenes of the S,B in {{0.1,3,6,9}} grid x {runs} runs x {cycles} "
                      f"periods (pure-Python Philox simulator); {workers} processes; {dt:.2f} s wall"}


def mc_sweep_workload(args):
    """The Monte Carlo validation of the model (Section 3.5): (b) S, B in
    {0.1, 3, 6, 9}, 100 runs x 50,000 periods at 2^10 bins, against the
    model at 2^5..2^10 bins; (c) S, B over [0, 10] (levels 0.1, 1..10), 25
    runs x 50,000 periods at 2^8 bins.  Dead time 75 ns, period 100 ns,
    pulse at 30 ns with sigma 0.5 ns.  One step = both simulations and the
    float64 model solves for all (S, B, N), on the GPU."""
    import numpy as np
    import torch

    from paper_2509_20500_amd import dtm
    from synth import scenes as sc

    cycles, burn = 50_000, 100
    e2 = sc.paper_grid(dead_time=75.0, n_bins=1024)
    e3 = sc.paper_rmse_grid(n_bins=256, dead_time=75.0)
    levels = [2 ** k for k in range(5, 11)]
    model = np.concatenate([sc.paper_grid(dead_time=75.0, n_bins=nb) for nb in levels] + [e3])
    plans, keep = [], []
    for scenes, opts in ((e2, dtm.opts(tol=1e-10)), (e3, dtm.opts(tol=1e-10)), (model, dtm.opts(tol=1e-12))):
        pl = dtm.Plan(scenes, "f64", opts)
        ws = torch.empty(pl.workspace_bytes, dtype=torch.uint8, device="cuda")
        pl.bind(ws)
        plans.append(pl)
        keep.append(ws)
    p2, p3, pm = plans
    h2 = torch.empty(p2.pi_elems, dtype=torch.int32, device="cuda")
    h3 = torch.empty(p3.pi_elems, dtype=torch.int32, device="cuda")
    o2 = torch.zeros(p2.n_pixels, dtype=torch.int32, device="cuda")
    o3 = torch.zeros(p3.n_pixels, dtype=torch.int32, device="cuda")
    pi = torch.empty(pm.pi_elems, dtype=torch.float64, device="cuda")
    infos = torch.zeros(pm.n_pixels * 40, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    mc_ms = []

    def step(record=False):
        if record:
            ev[0].record(stream)
        p2.mc_histograms(100, cycles, burn, 2509, hist=h2, over=o2)
        if record:
            ev[1].record(stream)
            ev[2].record(stream)
        p3.mc_histograms(25, cycles, burn, 20500, hist=h3, over=o3)
        if record:
            ev[3].record(stream)
        pm.solve(pi, infos)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        step(record=True)
        torch.cuda.synchronize()  # per-launch events are read after each step
        mc_ms.append((ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])))
    end.record(stream)
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(end) / args.steps
    periods = cycles * (100 * p2.n_pixels + 25 * p3.n_pixels)
    k2 = float(np.mean([a for a, _ in mc_ms]))
    k3 = float(np.mean([b for _, b in mc_ms]))

    info = dtm.infos_to_numpy(infos)
    pis = pi.cpu().numpy()
    offm = pm.pi_offsets
    hist2 = h2.cpu().numpy().view(np.uint32).astype(np.float64)
    hist3 = h3.cpu().numpy().view(np.uint32).astype(np.float64)
    off2, off3 = p2.pi_offsets, p3.pi_offsets
    table = {}
    for li, nb in enumerate(levels):
        l1s, rms = [], []
        for q in range(p2.n_pixels):
            h = hist2[off2[q]:off2[q + 1]]
            hn = h.reshape(nb, 1024 // nb).sum(axis=1) / h.sum()
            k = li * p2.n_pixels + q
            d = pis[offm[k]:offm[k + 1]] - hn
            l1s.append(float(np.abs(d).sum()))
            rms.append(float(np.sqrt(np.mean(d * d))))
        table[str(nb)] = {"l1_mean": float(np.mean(l1s)), "l1_min": float(np.min(l1s)),
                          "l1_max": float(np.max(l1s)), "rmse_mean": float(np.mean(rms))}
    base = len(levels) * p2.n_pixels
    rmse3, noise3 = [], []
    for q in range(p3.n_pixels):
        h = hist3[off3[q]:off3[q + 1]]
        m = h.sum()
        hn = h / m
        d = pis[offm[base + q]:offm[base + q + 1]] - hn
        rmse3.append(float(np.sqrt(np.mean(d * d))))
        noise3.append(float(np.sqrt(np.mean(hn * (1.0 - hn) / m))))
    rmse3, noise3 = np.array(rmse3), np.array(noise3)

    # Discretisation variants of the model against the same Monte Carlo
    # histograms (after the timed region; factored float64 solves).
    variants = {}
    vflags = {"shift_nearest": dtm.DTM_FLAG_SHIFT_NEAREST, "shift_interp": dtm.DTM_FLAG_SHIFT_INTERP,
              "lambda_bin_mean": dtm.DTM_FLAG_LAMBDA_BIN_MEAN, "bin_integral": dtm.DTM_FLAG_BIN_INTEGRAL,
              "paper": 0}
    for name, fl in vflags.items():
        o = dtm.opts(tol=1e-12)
        o.flags |= fl | dtm.DTM_FLAG_NO_DENSE
        pv = dtm.Plan(model, "f64", o)
        wv = torch.empty(pv.workspace_bytes, dtype=torch.uint8, device="cuda")
        pv.bind(wv)
        piv = torch.empty(pv.pi_elems, dtype=torch.float64, device="cuda")
        infv = torch.zeros(pv.n_pixels * 40, dtype=torch.uint8, device="cuda")
        pv.solve_factored(piv, infv)
        torch.cuda.synchronize()
        pvs = piv.cpu().numpy()
        ov_ = pv.pi_offsets
        l1n = {}
        for li, nb in enumerate(levels):
            l1s = []
            for q in range(p2.n_pixels):
                h = hist2[off2[q]:off2[q + 1]]
                hn = h.reshape(nb, 1024 // nb).sum(axis=1) / h.sum()
                k = li * p2.n_pixels + q
                l1s.append(float(np.abs(pvs[ov_[k]:ov_[k + 1]] - hn).sum()))
            l1n[str(nb)] = float(np.mean(l1s))
        rm = []
        for q in range(p3.n_pixels):
            h = hist3[off3[q]:off3[q + 1]]
            d = pvs[ov_[base + q]:ov_[base + q + 1]] - h / h.sum()
            rm.append(float(np.sqrt(np.mean(d * d))))
        variants[name] = {"grid_4x4_l1_mean_by_bins": l1n, "grid_11x11_n256_rmse_mean": float(np.mean(rm)),
                          "all_converged": bool(np.all(dtm.infos_to_numpy(infv)["status"] == 0))}
        pv.close()
        del wv

    valu = profile_record("valu-record", "k_mc", "mc_sweep_e2", MC_SOURCES)
    out = {
        "metric": "Monte Carlo laser periods/s (model-validation sweeps, 2.31e8 periods per step)",
        "value": periods / (ms_step * 1e-3),
        "unit": "laser periods/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Section 3.5 validation: S,B in {0.1,3,6,9} x 100 runs x 50,000 periods "
                               "at 2^10 bins vs model at 2^5..2^10; S,B in {0.1,1..10} x 25 runs x 50,000 "
                               "periods at 2^8 bins; t_r 100 ns, t_d 75 ns, pulse 30 ns sigma 0.5 ns; "
                               "Philox4x32-10 streams; float64 model solves in the step",
                   "periods_per_step": periods},
        "roofline": {
            "bound": "alu", "unit": "G VALU wave-instructions/s", "peak": VALU_PEAK_G,
            "achieved": (valu / (k2 * 1e-3) / 1e9) if valu else None,
            "frac": (valu / (k2 * 1e-3) / 1e9 / VALU_PEAK_G) if valu else None,
            "traffic": None, "kernel": "k_mc + repair passes (S,B in {0.1,3,6,9} call)",
            "valu_insts_per_launch": valu,
        },
        "k_mc_ms": {"grid_4x4_n1024": k2, "grid_11x11_n256": k3},
        "model_vs_mc_grid_4x4": table,
        "model_vs_mc_grid_11x11_n256": {"rmse_mean": float(rmse3.mean()), "rmse_max": float(rmse3.max()),
                                        "mc_noise_rmse_mean": float(noise3.mean()),
                                        "rmse_over_noise_max": float((rmse3 / noise3).max())},
        "model_variants_vs_mc": variants,
        "overflow_pixels": int(o2.sum().item() + o3.sum().item()),
        "model_all_converged": bool(np.all(info["status"] == 0)),
    }
    for pl in plans:
        pl.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = mc_cpu_baseline(e2)
    return out


def spectral_workload(args):
    """Section 4's spectral analysis on the GPU: for S, B in {0.1, 1, ..., 10}
    at dead times 75 and 95 ns (242 pixels, N = 1024, period 100 ns, pulse at
    30 ns with sigma 0.5 ns), lambda_2 (gap and phase) and the empirical
    mixing steps to a total-variation distance of 0.25.  One step = one
    dtm_spectral_batched call (factored float64 operator, no matrix)."""
    import numpy as np
    import torch

    from oracle import dtm as odtm, spectral as ospec
    from paper_2509_20500_amd import dtm
    from synth import scenes as sc

    grids = [sc.paper_rmse_grid(n_bins=1024, dead_time=td) for td in (75.0, 95.0)]
    scenes = np.concatenate(grids)
    o = dtm.opts(tol=1e-12)
    o.flags |= dtm.DTM_FLAG_NO_DENSE
    plan = dtm.Plan(scenes, "f64", o)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    eps = 0.25
    scratch = torch.empty(plan.spectral_scratch_bytes(True), dtype=torch.uint8, device="cuda")
    out = torch.zeros(plan.n_pixels * dtm.SPECTRAL_INFO_BYTES, dtype=torch.uint8, device="cuda")
    ms = timed(lambda: plan.spectral(out, scratch, eps, 10000), args.steps, args.warmup)
    res = dtm.spectral_to_numpy(out)
    plan.close()
    n = 1024
    # algorithmic flops: each start state's distribution (kept on chip, one
    # wavefront per state) costs about 8 float64 operations per bin per step
    # (divide by S, two scan adds, the product, the distance to pi); counted
    # for the pixel's mixing steps, which bounds what the per-state stop runs
    alg_flops = float(np.sum(8.0 * n * n * np.maximum(res["mixing_steps"], 0)))
    # sampled check against LAPACK eigenvalues of the oracle's dense matrix
    rng = np.random.default_rng(0)
    worst = 0.0
    n_check = 8 if args.check is None else min(args.check, len(scenes))
    for p in rng.choice(len(scenes), n_check, replace=False):
        lam, third = ospec.second_eigenvalue(odtm.transition_matrix(scenes[p]))
        worst = max(worst, abs(res["lambda2_abs"][p] - abs(lam)))
    dynamics = {"td75": single_bin_dynamics(scenes, res, grid=0),
                "td95": single_bin_dynamics(scenes, res, grid=1)}
    summary = {}
    for g, td in zip(range(2), (75.0, 95.0)):
        r = res[g * 121:(g + 1) * 121]
        B = grids[g]["background_flux"]
        gap = 1.0 - r["lambda2_abs"]
        # the gap as B grows, at each S: fraction of S rows where it shrinks
        gs = gap.reshape(11, 11)
        summary[f"td{int(td)}"] = {
            "gap_min": float(gap.min()), "gap_max": float(gap.max()),
            "gap_decreases_with_B_rows": int(np.sum(gs[:, -1] < gs[:, 0])),
            "corr_gap_B": float(np.corrcoef(gap, B)[0, 1]),
            "phase_min": float(r["lambda2_arg"].min()), "phase_max": float(r["lambda2_arg"].max()),
            "frac_phase_below_0.1": float(np.mean(r["lambda2_arg"] < 0.1)),
            "corr_phase_B": float(np.corrcoef(r["lambda2_arg"], B)[0, 1]),
            "mixing_steps_min": int(r["mixing_steps"].min()), "mixing_steps_max": int(r["mixing_steps"].max()),
        }
    return {
        "metric": "spectral analysis pixels/s (lambda_2 and mixing steps, N=1024)",
        "value": plan.n_pixels / (ms * 1e-3), "unit": "pixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "S,B in {0.1,1..10} x t_d in {75,95} ns (242 pixels), N=1024, t_r 100 ns, "
                               "pulse 30 ns sigma 0.5 ns; lambda_2 and |lambda_3| by orthogonal iteration "
                               "(six vectors, Rayleigh-Ritz) on the deflated factored operator, mixing "
                               "steps to TV 0.25 from all 1024 start states",
                   "pixels": int(len(scenes))},
        "roofline": {"bound": "alu", "achieved": alg_flops / (ms * 1e-3) / 1e12, "peak": 78.6,
                     "unit": "TFLOP/s", "frac": alg_flops / (ms * 1e-3) / 1e12 / 78.6, "traffic": None,
                     "kernel": "k_mixing_wave", "alg_flops_per_launch": alg_flops,
                     "time": "whole call (k_spectral + k_mixing_wave)"},
        "lambda2_abs_vs_lapack_sampled_max": worst,
        "section4": summary,
        "single_bin_dynamics": dynamics,
    }


def fit_recurrence(e):
    """Least-squares two-term recurrence e[t+1] = a e[t] + c e[t-1] over a
    deviation sequence, each equation scaled by the size of its right-hand
    terms (the sequence decays by orders of magnitude); returns the modulus
    and argument of the larger root of z^2 = a z + c (the per-sweep decay
    and rotation it follows)."""
    import numpy as np
    X = np.stack([e[1:-1], e[:-2]], axis=1)
    w = 1.0 / np.maximum(np.abs(X).max(axis=1), 1e-300)
    a, c = np.linalg.lstsq(X * w[:, None], e[2:] * w, rcond=None)[0]
    roots = np.roots([1.0, -a, -c])
    z = roots[np.argmax(np.abs(roots))]
    return float(abs(z)), float(abs(np.angle(z)))


def single_bin_dynamics(scenes, res, grid, sweeps=40, cells=None):
    """Section 4's single-bin view: for three pixels of one dead-time grid,
    chosen among those with |lambda_2| >= 0.5 (slow enough to leave tens of
    sweeps above float64 round-off): the smallest gap, then the largest and
    the smallest phase among the others.  Reports the deviation of the peak bin of the
    iterate from pi after t = 1 .. sweeps float64 power sweeps from uniform
    (batched dense solver, stopped after exactly t sweeps), and the decay and
    rotation per sweep that a two-term recurrence fitted to it follows,
    beside |lambda_2| and arg lambda_2 from the spectral call."""
    import numpy as np
    import torch

    from paper_2509_20500_amd import dtm
    lo, hi = grid * 121, (grid + 1) * 121
    r = res[lo:hi]
    if cells is None:
        slow = np.flatnonzero(r["lambda2_abs"] >= 0.5)
        if slow.size == 0:
            slow = np.arange(len(r))
        arg = r["lambda2_arg"][slow]
        cells = []
        for order in (np.argsort(-r["lambda2_abs"][slow], kind="stable"),
                      np.argsort(-arg, kind="stable"), np.argsort(arg, kind="stable")):
            pick = next((int(slow[i]) for i in order if int(slow[i]) not in cells), None)
            if pick is not None:
                cells.append(pick)
    sel = scenes[lo:hi][cells]
    traj = []
    for t in range(1, sweeps + 1):
        o = dtm.opts(tol=1e-300, max_iter=t, stop_rule=dtm.DTM_STOP_CHANGE)
        plan = dtm.Plan(sel, "f64", o)
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
        plan.bind(ws)
        pi = torch.empty(plan.pi_elems, dtype=torch.float64, device="cuda")
        infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
        plan.solve(pi, infos)
        torch.cuda.synchronize()
        traj.append(pi.cpu().numpy())
        off = plan.pi_offsets
        plan.close()
    plan = dtm.Plan(sel, "f64", dtm.opts(tol=1e-13))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    pi = torch.empty(plan.pi_elems, dtype=torch.float64, device="cuda")
    infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    plan.solve(pi, infos)
    torch.cuda.synchronize()
    pis = pi.cpu().numpy()
    plan.close()
    out = []
    for q, cell in enumerate(cells):
        p_q = pis[off[q]:off[q + 1]]
        b = int(np.argmax(p_q))
        e = np.array([x[off[q] + b] for x in traj]) - p_q[b]
        keep = np.flatnonzero(np.abs(e) > 1e-9 * p_q[b])  # above float64 round-off
        e_fit = e[: keep[-1] + 1] if keep.size else e[:0]
        e_fit = e_fit[5:]  # past the first sweeps, where faster modes still show
        fit = fit_recurrence(e_fit) if e_fit.size >= 6 else (None, None)
        out.append({"S": float(sel[q]["signal_flux"]), "B": float(sel[q]["background_flux"]),
                    "dead_time_ns": float(sel[q]["dead_time_ns"]), "bin": b,
                    "lambda2_abs": float(r["lambda2_abs"][cell]), "lambda2_arg": float(r["lambda2_arg"][cell]),
                    "fit_decay_per_sweep": fit[0], "fit_rotation_per_sweep": fit[1],
                    "sweeps_fitted": int(e_fit.size),
                    "deviation": [float(v) for v in e[:12]]})
    return out


def single_pixel_workload(args):
    """The single-pixel configurations: N=1000 float64 to change < 1e-12
    (period 100 ns, sigma 0.5 ns at 30 ns, S 0.5, B 0.1, dead time 75 ns),
    and N=4096 at dead times {10, 33, 75, 150} ns for eight seeded scenes
    (seed 2), float64 and float32.  One step = dtm_build_transition +
    dtm_stationary_pdf of one pixel (host polling); the 4096-bin sweep points
    are also solved as one batched plan for comparison."""
    import numpy as np
    import torch

    from oracle import dtm as odtm
    from paper_2509_20500_amd import dtm
    from synth import scenes as sc

    def solve_one(s, dt, o, P, ws, pi):
        dtm.build_transition(s, P, ws)
        return dtm.stationary_pdf(P, pi, ws, o)

    res = {}
    # N = 1000, float64, change < 1e-12
    s1 = sc.single_pixel_n1000()
    n = 1000
    P = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ws = dtm.workspace(n, "f64")
    pi = torch.empty(n, dtype=torch.float64, device="cuda")
    o1 = dtm.opts(tol=1e-12, stop_rule=dtm.DTM_STOP_CHANGE, max_iter=100000)
    for _ in range(args.warmup):
        solve_one(s1, "f64", o1, P, ws, pi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = solve_one(s1, "f64", o1, P, ws, pi)
    torch.cuda.synchronize()
    ms1 = (time.perf_counter() - t0) * 1e3 / args.steps
    err1 = float(np.abs(pi.cpu().numpy() - odtm.stationary_solve(odtm.transition_matrix(s1))).sum())
    res["n1000_f64"] = {"ms_per_pixel": ms1, "sweeps": int(info.iterations), "l1_vs_oracle": err1}
    # N = 4096 sweep points
    scenes = sc.single_pixel_n4096()
    n = 4096
    refs = [odtm.stationary_solve(odtm.transition_matrix(s)) for s in scenes[:4 if args.check is None else args.check]]
    for dt, o in (("f64", dtm.opts(tol=1e-10)), ("f32", dtm.opts(tol=1e-6))):
        tdt = torch.float64 if dt == "f64" else torch.float32
        P = torch.empty((n, n), dtype=tdt, device="cuda")
        ws = dtm.workspace(n, dt)
        pi = torch.empty(n, dtype=tdt, device="cuda")
        solve_one(scenes[0], dt, o, P, ws, pi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        errs, sweeps = [], []
        for k, s in enumerate(scenes):
            info = solve_one(s, dt, o, P, ws, pi)
            sweeps.append(info.iterations)
            if k < len(refs):
                errs.append(float(np.abs(pi.cpu().numpy().astype(np.float64) - refs[k]).sum()))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / len(scenes)
        del P
        plan = dtm.Plan(scenes, dt, o)
        wsb = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
        plan.bind(wsb)
        pib = torch.empty(plan.pi_elems, dtype=tdt, device="cuda")
        infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
        plan.solve(pib, infos)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            plan.solve(pib, infos)
        torch.cuda.synchronize()
        msb = (time.perf_counter() - t1) * 1e3 / args.steps
        got = pib.cpu().numpy().astype(np.float64)
        off = plan.pi_offsets
        errb = max(float(np.abs(got[off[k]:off[k + 1]] - refs[k]).sum()) for k in range(len(refs)))
        plan.close()
        del wsb
        res[f"n4096_{dt}"] = {"ms_per_pixel_single_path": ms, "mean_sweeps": float(np.mean(sweeps)),
                              "l1_vs_oracle_max": max(errs) if errs else None,
                              "batched_ms_all_sweep_points": msb, "batched_pixels": len(scenes),
                              "batched_l1_vs_oracle_max": errb}
    return {
        "metric": "single-pixel stationary PDF latency (N=1000 float64 to change < 1e-12)",
        "value": 1e3 / ms1, "unit": "pixels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "single pixels: N=1000 float64 (t_d 75 ns, sigma 0.5 ns at 30 ns, S 0.5, B 0.1); "
                               "N=4096 sigma 0.2 ns, t_d in {10,33,75,150} ns x 8 seeded scenes (seed 2), "
                               "float64 and float32"},
        "single_pixel": res,
    }


def _oracle_one(rec):
    import numpy as np

    from oracle import dtm as odtm
    from synth.scenes import make_scenes
    s = make_scenes(*rec)
    return float(np.sum(odtm.stationary_solve(odtm.transition_matrix(s))))


def _oracle_power_one(rec):
    """The oracle's vectorised build and its power iteration (BLAS
    vector-matrix products) from uniform to an L1 change below 1e-9."""
    from oracle import dtm as odtm
    from synth.scenes import make_scenes
    s = make_scenes(*rec)
    x, _, _ = odtm.stationary_power(odtm.transition_matrix(s), tol_change=1e-9)
    return float(x.sum())


def _noop(_):
    return 0


def cpu_baseline(scenes, sample):
    """The float64 oracle (dense build + LAPACK solve) on a bounded sample of
    the same pixels, one process per host core (capped at 16), one BLAS
    thread each."""
    import multiprocessing as mp
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    workers = max(1, min(os.cpu_count() or 1, 16))
    recs = [(float(s["period_ns"]), float(s["dead_time_ns"]), float(s["pulse_center_ns"]),
             float(s["pulse_sigma_ns"]), float(s["signal_flux"]), float(s["background_flux"]),
             int(s["n_bins"])) for s in scenes[:sample]]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_noop, range(workers))
        pool.map(_oracle_one, recs[:workers])  # imports and page-in outside the clock
        t0 = time.perf_counter()
        pool.map(_oracle_one, recs, chunksize=max(1, len(recs) // (4 * workers)))
        dt = time.perf_counter() - t0
        pool.map(_oracle_power_one, recs[:workers])
        t0 = time.perf_counter()
        pool.map(_oracle_power_one, recs, chunksize=max(1, len(recs) // (4 * workers)))
        dt_pow = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": len(recs) / dt, "unit": "pixels/s", "cores": workers, "kind": "oracle",
        "sample": f"first {len(recs)} pixels of the workload; float64 dense build + LAPACK solve; "
                  f"{workers} processes x 1 BLAS thread; {dt:.2f} s wall",
        "host": {"cpu_count": os.cpu_count(), "cpu_model": model},
        "power_iteration": {
            "value": len(recs) / dt_pow, "unit": "pixels/s",
            "sample": "the same pixels and processes; the oracle's vectorised build + power iteration "
                      f"(BLAS vector-matrix products) from uniform to an L1 change < 1e-9; {dt_pow:.2f} s wall",
        },
    }


def plain_single_pixel(scenes, sample=256):
    """The plain single-pixel GPU path on the first `sample` pixels: per
    pixel one dtm_build_transition and one dtm_stationary_pdf (float32, the
    same stop rule and 1e-6 target, host polling), one pixel after another."""
    import numpy as np
    import torch

    from paper_2509_20500_amd import dtm
    n = int(scenes["n_bins"][0])
    P = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ws = dtm.workspace(n, "f32")
    pi = torch.empty(n, dtype=torch.float32, device="cuda")
    o = dtm.opts(tol=1e-6)
    dtm.build_transition(scenes[0], P, ws)
    dtm.stationary_pdf(P, pi, ws, o)
    torch.cuda.synchronize()
    sweeps = []
    t0 = time.perf_counter()
    for s in scenes[:sample]:
        dtm.build_transition(s, P, ws)
        info = dtm.stationary_pdf(P, pi, ws, o)
        if info.status != dtm.DTM_OK:
            raise RuntimeError(f"single-pixel solve failed: {info.status}")
        sweeps.append(info.iterations)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"pixels_per_s": sample / dt, "sample": f"first {sample} pixels, one build + one solve each",
            "mean_sweeps": float(np.mean(sweeps))}


def copy_calibration(nbytes=1 << 30, reps=10):
    """A plain device-to-device copy of known size (torch's elementwise copy
    kernel): its achieved GB/s, and the reference whose FETCH_SIZE and
    WRITE_SIZE counters (nbytes each per launch) scale the solver's."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    return {"bytes_read": nbytes, "bytes_written": nbytes, "ms": ms,
            "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def probe_lib():
    """The bandwidth probe's own library (built beside libdtm.so, not part of
    the method's C-ABI)."""
    import ctypes
    path = os.path.join(ROOT, "paper_2509_20500_amd", "libdtm_probe.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build with `python -m paper_2509_20500_amd.build`")
    L = ctypes.CDLL(path)
    P, I32 = ctypes.c_void_p, ctypes.c_int32
    L.dtm_stream_probe.restype = ctypes.c_int
    L.dtm_stream_probe.argtypes = [P, ctypes.c_size_t, I32, I32, P, P]
    return L


def pattern_ceiling(n_chunks, chunk_bytes, passes, reps=3):
    """GB/s of the dense solver's access pattern without its arithmetic
    (dtm_stream_probe): every chunk written once in one launch, then read
    back in a second; the time for `passes` (fractional) reads is
    interpolated between the whole numbers around it."""
    import math

    import torch

    from paper_2509_20500_amd import dtm
    probe = probe_lib()
    buf = torch.empty(n_chunks * chunk_bytes, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    lo = max(0, int(math.floor(passes)))
    ms = {}
    for r in (lo, lo + 1):
        def run():
            dtm.check(probe.dtm_stream_probe(buf.data_ptr(), chunk_bytes, n_chunks, r, sink.data_ptr(),
                                             dtm._stream(None)), "dtm_stream_probe")
        ms[r] = timed(run, reps, 1)
    f = passes - lo
    t = ms[lo] + f * (ms[lo + 1] - ms[lo])
    del buf
    return {"gbs": n_chunks * chunk_bytes * (1.0 + passes) / (t * 1e-3) / 1e9, "chunks": n_chunks,
            "chunk_bytes": chunk_bytes, "reads": passes, "ms": t}


def host_inclusive(scenes, dtype, sopts, tiles, ws, reps=3):
    """The headline step with the host in the loop: plan from the host scene
    array (validation, offsets, launch shapes), bind (metadata upload, which
    synchronises), solve, then pi and infos copied over PCIe into pinned host
    buffers.  The caller-owned workspace is reused; wall clock, median of
    reps after one warm-up."""
    import time

    import numpy as np
    import torch

    from paper_2509_20500_amd import dtm
    tdt = torch.float32 if dtype == "f32" else torch.float64
    times = []
    pi_h = infos_h = None
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = dtm.Plan(scenes, dtype, sopts, tiles)
        plan.bind(ws)
        pi = torch.empty(plan.pi_elems, dtype=tdt, device="cuda")
        infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
        if pi_h is None:
            pi_h = torch.empty(plan.pi_elems, dtype=tdt, pin_memory=True)
            infos_h = torch.empty(plan.n_pixels * 40, dtype=torch.uint8, pin_memory=True)
        plan.solve(pi, infos)
        pi_h.copy_(pi, non_blocking=True)
        infos_h.copy_(infos, non_blocking=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan.close()
        if r:
            times.append(t1 - t0)
    t = float(np.median(times))
    return {"value": len(scenes) / t, "unit": "pixels/s", "ms": t * 1e3,
            "what": "plan from host scenes + bind (metadata upload) + solve + pi and infos to pinned host memory",
            "pi_bytes_to_host": int(pi_h.numel() * pi_h.element_size())}


def timed(step, steps, warmup):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(stream)
    for _ in range(steps):
        step()
    e.record(stream)
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


def warm_start_workload(args):
    """The learned warm start at N=1024: train the network on 200,000 PDFs the
    solver produces from uniform-workload sampling (seed 5), its logits added
    to the log of the flux start lambda / sum(lambda) (the network learns a
    correction to the method's own start), then solve 4,096 held-out pixels
    (seed 6) from uniform, from the flux start and from the network's
    prediction.  The timed warm step includes the feature and prior kernels
    and the network's forward pass."""
    import numpy as np
    import torch

    from oracle import pool as opool
    from paper_2509_20500_amd import dtm
    from paper_2509_20500_amd.warmstart import WarmStartMLP, _bind, solve_targets
    from synth import scenes as sc

    t0 = time.perf_counter()
    train = sc.warm_start_train()
    targets, tinfo = solve_targets(train)
    targets = (targets / targets.sum(dim=1, keepdim=True)).contiguous()
    t_targets = time.perf_counter() - t0
    print(f"warm_start: {train.size} training targets in {t_targets:.1f} s", file=sys.stderr, flush=True)
    net = WarmStartMLP(max_batch=1024, seed=0, zero_output=True)
    feat, shift = net.features(train)
    prior = net.flux_prior(train)
    t1 = time.perf_counter()
    hist = net.fit(feat, targets, epochs=args.epochs, lr=3e-3, prior=prior, shift=shift)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    print(f"warm_start: {args.epochs} epochs in {t_train:.1f} s, loss {hist[0]:.3f} -> {hist[-1]:.3f}",
          file=sys.stderr, flush=True)
    del targets, feat, prior, shift

    held = sc.warm_start_eval()
    flux_opts = dtm.opts(tol=1e-6)
    flux_opts.flags |= dtm.DTM_FLAG_START_FLUX
    plan = dtm.Plan(held, "f32", dtm.opts(tol=1e-6))
    plan_f = dtm.Plan(held, "f32", flux_opts)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    ws_f = torch.empty(plan_f.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    plan_f.bind(ws_f)
    pi_u = torch.empty(plan.pi_elems, dtype=torch.float32, device="cuda")
    pi_f = torch.empty_like(pi_u)
    pi_w = torch.empty_like(pi_u)
    inf_u = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    inf_f = torch.zeros_like(inf_u)
    inf_w = torch.zeros_like(inf_u)
    raw = torch.from_numpy(np.ascontiguousarray(held).view(np.uint8).copy()).cuda()
    feat_h = torch.empty((plan.n_pixels, 5), dtype=torch.float32, device="cuda")
    shift_h = torch.empty(plan.n_pixels, dtype=torch.int32, device="cuda")
    prior_h = torch.empty((plan.n_pixels, 1024), dtype=torch.float32, device="cuda")
    x0 = torch.empty((plan.n_pixels, 1024), dtype=torch.float32, device="cuda")
    net_lib = _bind()

    def warm_step():
        st = dtm._stream(None)
        dtm.check(net_lib.dtm_mlp_features(raw.data_ptr(), plan.n_pixels, feat_h.data_ptr(), shift_h.data_ptr(),
                                           st))
        dtm.check(net_lib.dtm_mlp_flux_prior(raw.data_ptr(), plan.n_pixels, prior_h.data_ptr(), st))
        for a in range(0, plan.n_pixels, net.max_batch):
            b = min(plan.n_pixels, a + net.max_batch)
            dtm.check(net_lib.dtm_mlp_forward(net.ws.data_ptr(), net.max_batch, feat_h[a:b].data_ptr(),
                                              prior_h[a:b].data_ptr(), shift_h[a:b].data_ptr(), b - a,
                                              x0[a:b].data_ptr(), st))
        plan.solve(pi_w, inf_w, x0.view(-1))

    ms_u = timed(lambda: plan.solve(pi_u, inf_u), args.steps, args.warmup)
    ms_f = timed(lambda: plan_f.solve(pi_f, inf_f), args.steps, args.warmup)
    ms_w = timed(warm_step, args.steps, args.warmup)
    iu, i_f, iw = (dtm.infos_to_numpy(t) for t in (inf_u, inf_f, inf_w))
    off = plan.pi_offsets
    plan.close()
    plan_f.close()
    del ws, ws_f

    # correctness gate outside the timed region: every held-out pixel of the
    # three runs against the float64 oracle (one oracle solve per pixel)
    t_check = time.perf_counter()
    refs = opool.stationary_many(held)
    t_check = time.perf_counter() - t_check
    l1 = {}
    for name, t in (("uniform", pi_u), ("flux", pi_f), ("warm", pi_w)):
        v = t.cpu().numpy().astype(np.float64)
        l1[name] = np.array([np.abs(v[off[p]:off[p + 1]] - refs[p]).sum() for p in range(len(held))])
    pu = pi_u.cpu().numpy().astype(np.float64)
    x0n = x0.cpu().numpy().astype(np.float64).reshape(-1)
    start_l1 = float(np.mean([np.abs(x0n[off[p]:off[p + 1]] - pu[off[p]:off[p + 1]]).sum()
                              for p in range(len(held))]))
    n = held["n_bins"].astype(np.float64)
    alg_w = float(np.sum(4 * n * n * iw["dense_sweeps"]))
    fallbacks = int(np.sum((iw["flags"] & (dtm.DTM_INFO_RESTARTED | dtm.DTM_INFO_WARM_REJECTED)) != 0))

    def start_report(ms, info, key):
        return {"pixels_per_s": len(held) / (ms * 1e-3), "ms_per_step": ms,
                "mean_sweeps": float(info["iterations"].mean()), "l1_vs_oracle_max": float(l1[key].max())}

    l1_all = max(float(v.max()) for v in l1.values())
    return {
        "metric": "stationary-PDF pixels/s at N=1024, L1<=1e-6 vs FP64 oracle; % HBM roofline",
        "value": len(held) / (ms_w * 1e-3),
        "unit": "pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_w,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "learned warm start at N=1024: MLP 5-256-256-1024 (GELU, bf16 GEMMs) whose "
                               "logits, in the frame of the pulse bin, correct the log flux start, softmax; "
                               "trained on 200,000 solver PDFs "
                               "(seed 5), 4,096 held-out pixels (seed 6); timed step = features + prior + "
                               "MLP forward + warm-started solve",
                   "pixels": len(held), "epochs": args.epochs},
        "roofline": {"bound": "hbm", "achieved": alg_w / (ms_w * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": alg_w / (ms_w * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_solve_build + k_solve_sweeps", "alg_bytes_per_launch": alg_w},
        "uniform_start": start_report(ms_u, iu, "uniform"),
        "flux_start": start_report(ms_f, i_f, "flux"),
        "warm_start": dict(start_report(ms_w, iw, "warm"), mean_l1_start_to_pi=start_l1, fallbacks=fallbacks),
        "speedup_vs_uniform": ms_u / ms_w,
        "speedup_vs_flux_start": ms_f / ms_w,
        "training": {"targets_s": t_targets, "train_s": t_train, "loss_first": hist[0], "loss_last": hist[-1],
                     "targets_all_converged": bool(np.all(tinfo["status"] == 0))},
        "all_converged": bool(np.all(iw["status"] == 0) and np.all(iu["status"] == 0)
                              and np.all(i_f["status"] == 0)),
        "l1_vs_oracle_max": l1_all,
        "l1_vs_oracle": {"max": l1_all, "pixels": len(held), "of": len(held), "sample": "every pixel, all three starts",
                         "oracle": "float64 dense build + LAPACK solve per pixel", "wall_s": t_check},
    }

def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", default="batched_uniform",
                    choices=["batched_uniform", "batched_uneven", "warm_start", "mc_sweep", "single_pixel",
                             "spectral"])
    ap.add_argument("--epochs", type=int, default=150, help="warm_start: training epochs")
    ap.add_argument("--pixels", type=int, default=0, help="0 = the workload's own count")
    ap.add_argument("--graph", action="store_true", help="replay the solve as a captured HIP graph")
    ap.add_argument("--solver", default="dense", choices=["dense", "factored"],
                    help="dense: the materialised matrix (headline); factored: O(n) sweeps, float64")
    ap.add_argument("--autotune", action="store_true", help="pick tile shapes by timing candidates")
    ap.add_argument("--check", type=int, default=None,
                    help="pixels compared with the float64 oracle after timing: 0 = every pixel (default "
                         "for the uniform batch), k > 0 = k sampled pixels (uniform batch) or k pixels of "
                         "each size (uneven batch, default 4)")
    ap.add_argument("--check-workers", type=int, default=0,
                    help="host processes of the oracle check (0 = one per core up to 16; 1 = in this process)")
    ap.add_argument("--cpu-sample", type=int, default=512)
    ap.add_argument("--single-sample", type=int, default=256,
                    help="pixels timed on the plain single-pixel GPU path (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--threads", type=int, default=0, help="one-block solver block size (0 = default)")
    ap.add_argument("--unroll", type=int, default=0, help="rows in flight per thread (0 = default)")
    ap.add_argument("--fused-max-bins", type=int, default=0, help="largest n of the one-block solver (0 = default)")
    ap.add_argument("--band-rows", type=int, default=0, help="rows per banded work item (0 = default)")
    ap.add_argument("--band-cpt", type=int, default=0, help="column vectors per thread, banded (0 = default)")
    ap.add_argument("--independent-paths", type=int, default=0, choices=[0, 1],
                    help="1: one-block and banded pixels sweep without waiting for each other's builds")
    ap.add_argument("--fused-blocks", type=int, default=0,
                    help="persistent workgroups of the one-block sweeps (0 = one per pixel)")
    ap.add_argument("--dense-sweeps", type=int, default=0,
                    help="sweeps of a pixel's dense matrix before the float64 continuation (0 = default)")
    ap.add_argument("--band-min-items", type=int, default=0,
                    help="banded sweeps stop, and their pixels continue in float64, once fewer work items "
                         "than this are left (0 = never)")
    ap.add_argument("--variant", default="paper",
                    choices=["paper", "nearest", "bin_mean", "bin_integral", "interp"],
                    help="discretisation of the model (interp needs --solver factored)")
    ap.add_argument("--start", default="flux", choices=["uniform", "flux"],
                    help="dense solver start vector: lambda / sum(lambda), the no-dead-time pi (default), "
                         "or uniform")
    ap.add_argument("--calibrate", action="store_true",
                    help="also time a plain 1 GiB device copy (the reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); pixels shard across GPUs "
              "with no communication, so the multi-GPU figure is the one-GPU figure times N.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_20500_amd import dtm
    from synth import scenes as sc

    dtm.lib()
    torch.cuda.set_device(0)
    if args.workload in ("warm_start", "mc_sweep", "single_pixel", "spectral"):
        out = {"warm_start": warm_start_workload, "mc_sweep": mc_sweep_workload,
               "single_pixel": single_pixel_workload, "spectral": spectral_workload}[args.workload](args)
        print(json.dumps(out), flush=True)
        return
    uneven = args.workload == "batched_uneven"
    if uneven:
        scenes = sc.batched_uneven(n_pixels=args.pixels or 2048)
    else:
        scenes = sc.batched_uniform(n_pixels=args.pixels or 4096)
    sopts = dtm.opts(tol=1e-6)
    tune_report = None
    if (args.threads or args.unroll or args.band_rows or args.band_cpt or args.fused_max_bins or args.dense_sweeps
            or args.independent_paths or args.fused_blocks or args.band_min_items):
        tiles = dtm.tiles(args.threads, args.unroll, args.fused_max_bins, args.band_rows, args.dense_sweeps,
                          args.band_cpt, args.independent_paths, args.fused_blocks, args.band_min_items)
    elif args.autotune:
        from paper_2509_20500_amd.autotune import autotune
        tiles, tune_report = autotune(scenes, args.dtype, sopts)
    else:
        tiles = None
    factored = args.solver == "factored"
    if factored:
        sopts.flags |= dtm.DTM_FLAG_NO_DENSE
    variant_flags = {"paper": 0, "nearest": dtm.DTM_FLAG_SHIFT_NEAREST, "bin_mean": dtm.DTM_FLAG_LAMBDA_BIN_MEAN,
                     "bin_integral": dtm.DTM_FLAG_BIN_INTEGRAL, "interp": dtm.DTM_FLAG_SHIFT_INTERP}
    if args.variant == "interp" and not factored:
        print("bench.py: the interpolated shift runs on the factored solver only (--solver factored)",
              file=sys.stderr)
        sys.exit(2)
    sopts.flags |= variant_flags[args.variant]
    if args.start == "flux":
        sopts.flags |= dtm.DTM_FLAG_START_FLUX
    plan = dtm.Plan(scenes, args.dtype, sopts, tiles)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    pi = torch.empty(plan.pi_elems, dtype=tdt, device="cuda")
    infos = torch.zeros(plan.n_pixels * 40, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    graph = plan.graph(pi, infos) if (args.graph and not factored) else None
    if factored:
        step = lambda: plan.solve_factored(pi, infos)  # noqa: E731
    else:
        step = graph.launch if graph else (lambda: plan.solve(pi, infos))

    progress(f"plan of {plan.n_pixels} pixels bound; {args.warmup} warmup steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        step()
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    ms_step = ms / args.steps
    progress(f"{args.steps} timed steps: {ms_step:.3f} ms per step")

    info = dtm.infos_to_numpy(infos)
    n = scenes["n_bins"].astype(np.float64)
    es = 4 if args.dtype == "f32" else 8
    # algorithmic bytes: each matrix written once; every sweep after the
    # first (taken while the matrix is built) reads it once.  A pixel
    # continued (or refined) in float64 reads its matrix only in the sweeps
    # before (the float64 sweeps regenerate it from its tables): the
    # report's dense_sweeps
    dense_passes = info["dense_sweeps"]
    alg_bytes = float(np.sum(es * n * n * dense_passes))
    achieved = alg_bytes / (ms_step * 1e-3) / 1e9
    value = plan.n_pixels / (ms_step * 1e-3)
    # factored sweeps: about 12 float64 operations per bin per sweep
    alg_flops = float(np.sum(12.0 * n * info["iterations"]))
    # counted VALU instructions of the factored launch on the headline pixels
    fact_valu = (profile_record("valu-record", "k_solve_factored_wave", "batched_uniform_n1024_factored",
                                FACT_SOURCES)
                 if (factored and not uneven and plan.n_pixels == 4096 and args.variant == "paper"
                     and args.dtype == "f32") else None)

    # correctness gate, outside the timed region: every pixel of the uniform
    # batch against the float64 oracle (a pool of host-core processes); for
    # the uneven batch, `--check` pixels of each size (the dense oracle at
    # 8192 bins takes tens of seconds per pixel)
    from oracle import dtm as odtm
    from oracle import pool as opool
    got = pi.cpu().numpy().astype(np.float64)
    off = plan.pi_offsets
    vecs = [got[off[p]:off[p + 1]] for p in range(plan.n_pixels)]
    rng = np.random.default_rng(0)
    if uneven:
        per = 4 if args.check is None else args.check
        sample = np.sort(np.concatenate([
            rng.choice(np.flatnonzero(scenes["n_bins"] == size), min(per, int(np.sum(scenes["n_bins"] == size))),
                       replace=False) for size in np.unique(scenes["n_bins"])])) if per > 0 \
            else np.arange(plan.n_pixels)
        sample_desc = f"{per} pixels of each size" if per > 0 else "every pixel"
    else:
        per = 0 if args.check is None else args.check
        sample = (np.sort(rng.choice(plan.n_pixels, min(per, plan.n_pixels), replace=False)) if per > 0
                  else np.arange(plan.n_pixels))
        sample_desc = f"{sample.size} sampled pixels" if per > 0 else "every pixel"
    progress(f"oracle check of {sample.size} pixels")
    t_check = time.perf_counter()
    if args.variant == "paper":
        l1s = opool.l1_many(scenes[sample], [vecs[p] for p in sample], workers=args.check_workers or None)
    else:
        from oracle import variants as ovar
        shift_lam = {"nearest": ("nearest", "point"), "bin_mean": ("ceil", "bin_mean"),
                     "bin_integral": ("ceil", "bin_integral"), "interp": ("interp", "point")}[args.variant]
        sample = sample[:16]
        sample_desc = f"{sample.size} sampled pixels (model variant)"
        l1s = np.array([float(np.abs(vecs[p] - odtm.stationary_solve(
            ovar.transition_matrix_variant(scenes[p], *shift_lam))).sum()) for p in sample])
    t_check = time.perf_counter() - t_check
    progress(f"oracle check done in {t_check:.1f} s")
    l1_report = {"max": float(l1s.max()), "median": float(np.median(l1s)), "pixels": int(sample.size),
                 "of": int(plan.n_pixels), "sample": sample_desc,
                 "oracle": "float64 dense build + LAPACK solve per pixel", "wall_s": t_check}

    if uneven:
        desc = ("2048 pixels, N from {512,1024,2048,4096,8192} weighted 16:8:4:2:1, period U[50,200] ns, "
                "dead time period*U[0.2,1.5], sigma U[0.1,1] ns, depth U[5,period-5], "
                "S log-U[0.05,5], B log-U[0.01,1], seed 4; ")
    else:
        desc = ("64x64 pixels, N=1024 bins over 100 ns, dead time 50 ns, sigma 0.4 ns, "
                "depth U[5,95] ns, S log-U[0.05,5], B log-U[0.01,1], seed 3; ")
    desc += (f"{args.dtype} build+sweeps, float64 check, L1<=1e-6" if not factored else
             f"factored solver (no matrix, O(n) float64 sweeps), {args.dtype} output, L1<=1e-6")
    desc += "; HIP graph" if graph else ""
    desc += (("; start lambda/sum(lambda)" if args.start == "flux" else "; uniform start")
             if not factored else "")
    desc += f"; model variant {args.variant}" if args.variant != "paper" else ""
    out = {
        "metric": "stationary-PDF pixels/s at N=1024, L1<=1e-6 vs FP64 oracle; % HBM roofline",
        "value": value,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": desc,
            "pixels": plan.n_pixels,
            "n_bins": 1024 if not uneven else "512..8192",
            "tiles": plan.tiles.as_dict(),
            "graph": bool(graph),
        },
        "roofline": ({
            # VALU issue of the counted launch (the kernel is bound by its
            # float64 erfc/exp chains and wavefront scans, not by flops)
            "bound": "alu",
            "achieved": fact_valu / (ms_step * 1e-3) / 1e9,
            "peak": VALU_PEAK_G,
            "unit": "G VALU wave-instructions/s",
            "frac": fact_valu / (ms_step * 1e-3) / 1e9 / VALU_PEAK_G,
            "traffic": None,
            "kernel": "k_solve_factored_wave",
            "valu_insts_per_launch": fact_valu,
            "sweep_flops_frac_of_f64_peak": alg_flops / (ms_step * 1e-3) / 1e12 / 78.6,
        } if fact_valu else {
            "bound": "alu",
            "achieved": alg_flops / (ms_step * 1e-3) / 1e12,
            "peak": 78.6,
            "unit": "TFLOP/s",
            "frac": alg_flops / (ms_step * 1e-3) / 1e12 / 78.6,
            "traffic": None,
            "kernel": "k_solve_factored_wave" if int(scenes["n_bins"].max()) <= 1024 else "k_solve_factored",
            "alg_flops_per_launch": alg_flops,
        }) if factored else {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (measured_traffic("k_solve_build+k_solve_sweeps",
                                         f"batched_uniform_n1024_{args.dtype}_start_{args.start}")
                        if (not uneven and plan.n_pixels == 4096 and not graph and not tiles
                            and args.variant == "paper")
                        # the uneven batch: the bytes depend on the dense-sweep budget, the
                        # banded hand-off, and the split into one-block and banded pixels and
                        # their work items (band partial sums), not on the one-block workgroup
                        # shapes or on graph replay
                        else measured_traffic("k_solve_build+k_solve_sweeps+k_band_sweep",
                                              f"batched_uneven_{args.dtype}_start_{args.start}"
                                              f"_dense{plan.tiles.dense_sweeps}_fmax{plan.tiles.fused_max_bins}"
                                              f"_band{plan.tiles.band_rows}_cpt{plan.tiles.band_cpt}"
                                              f"_mi{plan.tiles.band_min_items}")
                        if (uneven and plan.n_pixels == 2048 and args.variant == "paper") else None),
            "kernel": ("k_solve_build + k_solve_sweeps" if not uneven
                       else "k_solve_build + k_solve_sweeps + k_band_sweep"),
            "alg_bytes_per_launch": alg_bytes,
        },
        "iterations": {"mean": float(info["iterations"].mean()), "max": int(info["iterations"].max()),
                       "min": int(info["iterations"].min())},
        "all_converged": bool(np.all(info["status"] == 0)),
        "refined_pixels": int(np.sum((info["flags"] & dtm.DTM_INFO_REFINED) != 0)),
        "continued_pixels": int(np.sum((info["flags"] & dtm.DTM_INFO_CONTINUED) != 0)),
        "max_residual_l1": float(info["residual_l1"].max()),
        "l1_vs_oracle_max": l1_report["max"],
        "l1_vs_oracle": l1_report,
    }
    if tune_report is not None:
        out["autotune"] = {"cached": tune_report["cached"], "ms": tune_report["ms"]}
    if graph:
        graph.close()
    plan.close()
    if not uneven and not factored and not graph:
        out["host_inclusive"] = host_inclusive(scenes, args.dtype, sopts, tiles, ws)
    del ws
    if not uneven and not factored and not graph and plan.n_pixels == 4096:
        # the same access pattern without arithmetic, for reading the roofline
        pc = pattern_ceiling(plan.n_pixels, 4 * 1024 * 1024 if args.dtype == "f32" else 8 * 1024 * 1024,
                             float(info["dense_sweeps"].mean()) - 1.0)
        pc["kernel_frac_of_pattern"] = achieved / pc["gbs"]
        out["pattern_ceiling"] = pc
    if args.calibrate:
        out["copy_calibration"] = copy_calibration()
    if not uneven and not factored and args.single_sample > 0:
        out["plain_single_pixel_gpu"] = plain_single_pixel(scenes, args.single_sample)
        out["plain_single_pixel_gpu"]["batched_speedup"] = value / out["plain_single_pixel_gpu"]["pixels_per_s"]
    if not args.no_cpu_baseline and not uneven and not factored:
        progress(f"CPU oracle baseline on {args.cpu_sample} pixels")
        out["cpu_baseline"] = cpu_baseline(scenes, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
