#!/usr/bin/env python3
"""Throughput of the hyperspectral DOT Born hot path on one MI355X.

One step = the whole hot path over one wavelength shard of the workload: the fields for every
source and detector at the shard's wavelengths (Algorithm 1 with a recycled deflation space, all
systems batched, complex FP32 Krylov with FP64 residual refinement to rel-res 1e-8, each restart
cycle replayed from a hipGraph), then Born J v, Born J^H w and the PaLS misfit value and gradient
(forward and adjoint) on those fields.  The default workload is the large one: the 128x128x64
grid with 64 sources + 64 detectors over 128 wavelengths 650-1000 nm, plus its three companion
grids (32x32x16, 48x48x24, 80x80x40) at the same wavelengths, solved with the main grid as one
batch (each grid's launches on a stream of its own, concurrently).  Its wavelengths are split into 8
shards of 16 (one GPU's share when the wavelengths are spread over eight GPUs); step i solves
shard i mod 8, so the default 8 timed steps cover the whole workload once.

Prints one JSON line.  value = RHS x wavelength solves per second of whole steps (every grid).
Also reported: the main grid's own rate, Born J v GFLOP/s, the roofline of the dominant kernel
(from a separate instrumented pass: HIP events inside the library on the solve stream; the
timed steps run with the instrumentation off, so the graph path is what they time), Born
rooflines, the plain per-system FP64 solver on a subsample, measured HBM copy bandwidth, and the
CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Solver settings of the batched path: deflation space k = 5, m - k = 10 Arnoldi steps per
# cycle, 40 shift-invariant Lanczos steps, FP32 inner solves to 3e-5 (the fastest region of a
# sweep over k, m - k, n, the inner tolerance and the batch size on one 16-wavelength shard of
# the 128x128x64 grid).
RECYCLE_K, RESTART_M, LANCZOS_N, INNER_TOL = 5, 15, 40, 3e-5

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0   # dense MFMA
N_JAC = 42                  # Jacobian block: 2 chromophore contrasts + 40 PaLS parameters

# Workloads: the main grid, its companion grids, wavelength shards, systems per batch.
WORKLOADS = {
    "large": dict(main="large", companions=("large_g32", "large_g48", "large_g80"), shards=8, max_batch=512,
                  text="large: 128x128x64 grid (1048576 voxels, h=2 mm), 64 sources + 64 detectors, 128 wavelengths "
                       "650-1000 nm, with the companion grids 32x32x16 (16+16), 48x48x24 (24+24) and 80x80x40 (32+32) "
                       "at the same wavelengths"),
    "medium": dict(main="medium", companions=(), shards=1, max_batch=0,
                   text="medium: 64x64x32 grid (131072 voxels, h=2 mm), 16 sources + 16 detectors, 32 wavelengths "
                        "650-900 nm"),
    "batch": dict(main="batch", companions=(), shards=1, max_batch=0,
                  text="batch: 64x64x32 grid (131072 voxels, h=2 mm), 32 sources + 32 detectors, 64 wavelengths "
                       "650-900 nm"),
    "diff": dict(main="diff", companions=(), shards=1, max_batch=1152,
                 text="diff: 96x96x48 grid (442368 voxels, h=2 mm), 24 sources + 24 detectors, 48 wavelengths "
                      "650-900 nm"),
    "tiny": dict(main="tiny", companions=(), shards=1, max_batch=0,
                 text="tiny: 16x16x8 grid (2048 voxels, h=2 mm), 4 sources + 4 detectors, 8 wavelengths 650-860 nm"),
}

# Calibrated HBM bytes per dispatch of the Arnoldi step kernels (FETCH_SIZE x 2 + WRITE_SIZE, the
# factors of a device copy of known size), keyed by workload.  They belong to the kernel sources
# with this SHA-256 (common.h, krylov_index.h, krylov_kernels.h, krylov_tiled.h) and to the launch shape
# TRAFFIC_TUNING; after any change of either the traffic is reported as null.
TRAFFIC_SOURCES_SHA256 = "ea2a412b68babc8261a5658dc07573b9bc6592c9961b0c35b440d362c874e740"
TRAFFIC_TUNING = {"step_presum": 16, "step_group": 2, "step_vx": 1, "step_order": 4, "step_pair": 2}
TRAFFIC_BYTES_PER_LAUNCH: dict = {   # workload -> kernel -> calibrated HBM bytes per launch (main grid)
    "large": {"k_step_pair_t<update>": 20738055511, "k_step_pair_t<dots>": 17695971737},
}


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("common.h", "krylov_index.h", "krylov_kernels.h", "krylov_tiled.h"):
        with open(os.path.join(ROOT, "paper_1410_0986_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_identity() -> dict:
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(wname: str, n_sys: int):
    """Unrecycled GMRES(30) of the FP64 oracle on a bounded sample of the same workload."""
    from threadpoolctl import threadpool_info

    import workloads
    from oracle import fields as ofields
    from oracle import model as omodel

    w = workloads.config(wname)
    lams = list(range(0, w.L, max(1, w.L // n_sys)))[:n_sys]
    t0 = time.perf_counter()
    iters = 0
    for l in lams:
        A = omodel.operator(w, l)
        _, it, rr = ofields.gmres(A, omodel.rhs(w, w.rhs_voxels[0]), tol=1e-8, m=30, max_iter=20000)
        iters += it
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": len(lams) / dt, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(lams)} system(s) (source 0 at wavelength indices {lams}) of the {wname} grid, "
                      f"unrecycled GMRES(30) FP64 to rel-res 1e-8 (scipy sparse matvec + numpy), {iters} iterations, "
                      f"{dt:.1f} s", **host_identity()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: one pass over every shard)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-system FP64 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-born-variants", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="run the launch-shape autotuners before timing")
    ap.add_argument("--tuning", default="",
                    help="launch-shape fields set before timing, e.g. step_order=3,step_group=2")
    ap.add_argument("--studies", action="store_true",
                    help="secondary measurements (heterogeneous forward, boundary/shift study, preconditioner, "
                         "compression, reconstruction) on the first shard")
    ap.add_argument("--no-profile-pass", action="store_true", help="skip the instrumented roofline pass")
    ap.add_argument("--cpu-sample", type=int, default=3, help="systems in the CPU oracle sample")
    ap.add_argument("--peaks-gib", type=float, default=8.0,
                    help="scratch of the peak probes (HBM streams, MFMA loops); 0: skip")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the hot path is measured on one GPU's share; see the sharding notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1410_0986_amd as hd
    import workloads

    cfg = WORKLOADS[args.config]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)     # default priority
    w = workloads.config(cfg["main"])
    S, D, L, N = w.S, w.D, w.L, w.N
    R = S + D
    n_shards = cfg["shards"]
    Ls = L // n_shards
    steps = args.steps if args.steps is not None else n_shards
    shard_idx = [np.arange(i * Ls, (i + 1) * Ls) for i in range(n_shards)]
    mains = [workloads.subset_lambdas(w, ix) if n_shards > 1 else w for ix in shard_idx]
    ops = [hd.Operator.from_workload(ws) for ws in mains]
    comp_w = [workloads.config(c) for c in cfg["companions"]]
    comp_ops = [[hd.Operator.from_workload(workloads.subset_lambdas(cw, ix)) for ix in shard_idx] for cw in comp_w]

    def solve_opts(max_batch, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH):
        return hd.SolveOptions(rel_tol=1e-8, restart_m=RESTART_M, recycle_k=RECYCLE_K, lanczos_n=LANCZOS_N,
                               precision=hd.PREC_MIXED, inner_tol=INNER_TOL, flags=flags, max_iter=5000,
                               max_batch=max_batch)

    opts = solve_opts(cfg["max_batch"])
    copts = solve_opts(1024)
    v = torch.from_numpy(workloads.born_v(w, dtype=np.float32)).to(dev)
    wv_all = workloads.born_w(w)
    p_true, dc_true = workloads.pals_truth(w)
    p_eval, dc_eval = workloads.pals_perturbed(w, p_true, dc_true)
    tune = {}
    if args.tuning:
        tune = {k: int(x) for k, x in (kv.split("=") for kv in args.tuning.split(","))}
        for o in ops + [c for cl in comp_ops for c in cl]:
            hd.set_tuning(o, **tune)

    with torch.cuda.stream(stream):
        phi = torch.empty((Ls, R, N), dtype=torch.complex64, device=dev)
        cphi = [torch.empty((Ls, cw.S + cw.D, cw.N), dtype=torch.complex64, device=dev) for cw in comp_w]
        mu_t = hd.pals_shape(ops[0], p_true, dtype=torch.float32, device=dev)

        solve_trials = born_trials = []
        if args.autotune:
            solve_trials = hd.autotune_solve(ops[0], w.rhs_voxels, opts, out=phi)
            log(f"autotune of the step kernels done ({len(solve_trials)} candidates)")
            hd.solve_fields(ops[0], w.rhs_voxels, opts, out=phi)
            born_trials = hd.autotune_born(ops[0], phi[:, :S], phi[:, S:], v)
            log(f"autotune of J v done ({len(born_trials)} candidates)")
            best = hd.get_tuning(ops[0])
            for o in ops[1:]:
                hd.set_tuning(o, **best)

        def step(i):
            sh = i % n_shards
            op = ops[sh]
            # the main grid and its companion grids in one batch (their launches run concurrently)
            res = hd.solve_fields_batch([(op, w.rhs_voxels, opts, phi)] +
                                        [(col[sh], cw.rhs_voxels, copts, cp)
                                         for cw, col, cp in zip(comp_w, comp_ops, cphi)])
            _, it, rel, st = res[0]
            crel = [r[2] for r in res[1:]]
            cit = [r[1] for r in res[1:]]
            y = hd.born_apply(op, phi[:, :S], phi[:, S:], v)
            wv = torch.from_numpy(wv_all[shard_idx[sh]]).to(torch.complex64).to(dev)
            g = hd.born_apply_adjoint(op, phi[:, :S], phi[:, S:], wv)
            # PaLS misfit and gradient: data of the true shape, evaluated at a perturbed point
            ebar = torch.from_numpy(dc_true @ mains[sh].extinction).to(dev).to(torch.float32)
            y_obs = (ebar[:, None, None] * hd.born_apply(op, phi[:, :S], phi[:, S:], mu_t[None])[0]).contiguous()
            dct = torch.tensor(dc_eval, requires_grad=True)
            pt = torch.tensor(p_eval, requires_grad=True)
            f = hd.BornMisfit.apply(dct, pt, op, phi[:, :S], phi[:, S:], y_obs)
            f.backward()
            return it, rel, st, crel, cit, y, g

        for i in range(args.warmup):
            step(i)
            log(f"warmup step {i + 1}/{args.warmup} done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, rels, crels, cits = [], [], [], []
        for i in range(steps):
            it, rel, st, crel, cit, _, _ = step(i)
            its.append(it)
            rels.append(rel)
            crels.extend(crel)
            cits.extend(cit)
            log(f"timed step {i + 1}/{steps} (shard {i % n_shards}) done")
        torch.cuda.synchronize()
        t1 = time.perf_counter()

        # per-grid rates on shard 0, graph path (not part of the timed steps)
        per_grid = {}
        torch.cuda.synchronize()
        ta = time.perf_counter()
        hd.solve_fields(ops[0], w.rhs_voxels, opts, out=phi)
        torch.cuda.synchronize()
        per_grid[f"{w.nx}x{w.ny}x{w.nz}"] = round(R * Ls / (time.perf_counter() - ta), 1)
        for cw, col, cp in zip(comp_w, comp_ops, cphi):
            ta = time.perf_counter()
            hd.solve_fields(col[0], cw.rhs_voxels, copts, out=cp)
            torch.cuda.synchronize()
            per_grid[f"{cw.nx}x{cw.ny}x{cw.nz}"] = round((cw.S + cw.D) * Ls / (time.perf_counter() - ta), 1)
        log("per-grid rates done")

        # instrumented pass (roofline): library HIP events around every Arnoldi step-kernel launch of
        # one main-grid shard solve, graph capture off while they are on
        prof = {}
        if not args.no_profile_pass:
            hd.profile_enable(True)
            hd.solve_fields(ops[0], w.rhs_voxels, opts, out=phi)
            torch.cuda.synchronize()
            prof = hd.profile_read()
            hd.profile_enable(False)
            log("instrumented pass done")

        # Born products alone on shard 0's fields: HIP events on this stream
        op0 = ops[0]
        wv0 = torch.from_numpy(wv_all[shard_idx[0]]).to(torch.complex64).to(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

        def timed(fn, nrep=20):
            fn()
            e0.record(stream)
            for _ in range(nrep):
                fn()
            e1.record(stream)
            e1.synchronize()
            return e0.elapsed_time(e1) / nrep

        jv_ms = timed(lambda: hd.born_apply(op0, phi[:, :S], phi[:, S:], v))
        jhw_ms = timed(lambda: hd.born_apply_adjoint(op0, phi[:, :S], phi[:, S:], wv0))
        log("born timing done")

        variants = {}
        if not args.no_born_variants:
            variants = born_variants(hd, torch, np, workloads, w, mains[0], phi, v, dev, timed)
            log("born variants done")

        studies = None
        if args.studies:
            studies = run_studies(hd, torch, np, workloads, mains[0], ops[0], opts, phi, dev, p_true, dc_true)

        plain = None
        if not args.no_plain:
            w1 = workloads.Workload(**{**mains[0].__dict__, "src_voxels": w.src_voxels[:1],
                                       "det_voxels": w.det_voxels[:0], "extra": {}})
            op1 = hd.Operator.from_workload(w1)
            po = hd.SolveOptions(rel_tol=1e-8, restart_m=RESTART_M, recycle_k=RECYCLE_K, lanczos_n=LANCZOS_N,
                                 precision=hd.PREC_FP64, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_PER_SYSTEM, max_iter=5000)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, pit, prel, pst = hd.solve_fields(op1, w1.rhs_voxels, po, device=dev)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            plain = {"solves_per_s": Ls / (tb - ta), "sample": f"1 right-hand side x {Ls} wavelengths (shard 0) of the "
                                                              f"{w.nx}x{w.ny}x{w.nz} grid",
                     "max_rel_res": float(prel.max()), "mean_iters": float(pit.mean())}
            # the batched path's rate on the same grid (shard 0, every right-hand side)
            log("plain path done")

    peaks = None
    if args.peaks_gib > 0:
        # achievable peaks from the library's probe kernels (HBM streams, read/write mix, MFMA loops)
        torch.cuda.synchronize()
        peaks = {k: (round(v, 1) if isinstance(v, float) else v) for k, v in hd.measure_peaks(dev, args.peaks_gib).items()}
        peaks["buffer_gib"] = args.peaks_gib
        log("peak probes done")

    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / steps
    sys_main = R * Ls
    sys_comp = sum((cw.S + cw.D) * Ls for cw in comp_w)
    solves_per_s = (sys_main + sys_comp) * steps / elapsed
    rel_all = max(float(np.max(r)) for r in rels + crels)
    it_main = float(np.mean(np.stack(its)))
    jv_flops = 8.0 * S * D * N * Ls

    roof = None
    if prof:
        name, (launches, kms, kbytes) = max(prof.items(), key=lambda kv: kv[1][1])
        achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
        traffic = None
        tuned = hd.get_tuning(ops[0])
        if kernel_sources_sha256() == TRAFFIC_SOURCES_SHA256 and all(tuned[k] == x for k, x in TRAFFIC_TUNING.items()):
            traffic = TRAFFIC_BYTES_PER_LAUNCH.get(args.config, {}).get(name)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "bytes/launch",
                # the same achieved rate against the probes' measured streams: read-only, and the
                # update kernel's own mix (ten vectors read, one written)
                "frac_of_measured_read": round(achieved / peaks["read_GBps"], 4) if peaks else None,
                "frac_of_measured_read10_write1": round(achieved / peaks["read10_write1_GBps"], 4) if peaks else None,
                "kernel": name, "launches": launches, "avg_launch_ms": round(kms / max(launches, 1), 4),
                "algorithmic_bytes_per_launch": kbytes / max(launches, 1),
                "source": "instrumented pass: one main-grid shard solve, HIP events on the solve stream",
                "all_step_kernels": {k: {"launches": a_, "ms": round(b_, 2),
                                         "GB/s": round(c_ / (b_ * 1e-3) / 1e9, 1) if b_ > 0 else 0.0}
                                     for k, (a_, b_, c_) in prof.items()}}
    field_bytes = (S + D) * N * Ls * 8
    born_roof = {
        "jv_fp32": {"ms": round(jv_ms, 4), "tflops": round(jv_flops / (jv_ms * 1e-3) / 1e12, 2),
                    "mfma_frac_fp32": round(jv_flops / (jv_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
                    "mfma_frac_of_measured_fp32": round(jv_flops / (jv_ms * 1e-3) / 1e12 / peaks["mfma_f32_TFLOPs"], 4)
                    if peaks else None,
                    "field_GBps": round(field_bytes / (jv_ms * 1e-3) / 1e9, 1),
                    "hbm_frac": round(field_bytes / (jv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "flop_convention": "8*S*D*N*L complex MACs (no 3M credit)"},
        "jhw_fp32": {"ms": round(jhw_ms, 4), "tflops": round(jv_flops / (jhw_ms * 1e-3) / 1e12, 2),
                     "mfma_frac_fp32": round(jv_flops / (jhw_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
                     "mfma_frac_of_measured_fp32": round(jv_flops / (jhw_ms * 1e-3) / 1e12 / peaks["mfma_f32_TFLOPs"], 4)
                     if peaks else None,
                     "field_GBps": round(field_bytes / (jhw_ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(field_bytes / (jhw_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    out = {
        "metric": "RHS x wavelength solves/sec at rel-res 1e-8 (+ Born Jv GFLOP/s), batched vs plain",
        "value": round(solves_per_s, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 Krylov + f64 refinement",
        "data": "synthetic (seeded)",
        "config": {"workload": cfg["text"],
                   "step": f"one wavelength shard ({Ls} of {L} wavelengths; {n_shards} shards, step i solves shard "
                           f"i mod {n_shards}): {sys_main} main-grid systems + {sys_comp} companion-grid systems in one "
                           "batch, then "
                           "J v, J^H w and the PaLS misfit gradient on the main grid",
                   "systems_per_step": sys_main + sys_comp,
                   "solver": f"batched recycled GMRES, m={RESTART_M}, k={RECYCLE_K}, n={LANCZOS_N}, mean shift, "
                             f"FP32 inner to {INNER_TOL:g}, max_batch {cfg['max_batch'] or 'all'}, restart cycles replayed "
                             "from hipGraphs",
                   "max_rel_res": rel_all, "mean_iters_main": it_main},
        "main_grid_solves_per_s_shard0": per_grid.get(f"{w.nx}x{w.ny}x{w.nz}"),
        "per_grid_solves_per_s_shard0": per_grid,
        "born_jv_gflops": round(jv_flops / (jv_ms * 1e-3) / 1e9, 1),
        "born_jv_ms": round(jv_ms, 4),
        "born_adjoint_ms": round(jhw_ms, 4),
        "born_roofline": born_roof,
        "born_variants": variants,
        "studies": studies,
        "plain_fp64": plain,
        "speedup_vs_plain": round(per_grid[f"{w.nx}x{w.ny}x{w.nz}"] / plain["solves_per_s"], 2) if plain else None,
        "roofline": roof,
        "peaks_measured": peaks,
        "peaks_spec": {"hbm_GBps": HBM_PEAK_GBS, "fp32_tflops": FP32_PEAK_TFLOPS, "fp64_tflops": FP64_PEAK_TFLOPS,
                       "bf16_tflops": BF16_PEAK_TFLOPS},
        "tuning": {**hd.get_tuning(ops[0]), "autotuned": bool(args.autotune), "solve_candidates": len(solve_trials),
                   "born_candidates": len(born_trials)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg["main"], args.cpu_sample)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


def born_variants(hd, torch, np, workloads, w, w_shard, phi, v, dev, timed):
    """Born J v variants: FP32 / split-BF16 / BF16-stored fields, one probe vector on every wavelength
    of the shard and the 42-column Jacobian block on two, each against the FP64 products of the same
    fields."""
    S, D, N = w.S, w.D, w.N
    vj = torch.from_numpy(workloads.born_v(w, n_v=N_JAC, seed=2024, dtype=np.float32)).to(dev)
    pad = lambda x, m: -(-x // m) * m
    out = {}
    for nv, vv, nl in (("1", v, w_shard.L), (str(N_JAC), vj, 2)):
        w2 = workloads.subset_lambdas(w_shard, np.arange(nl))
        op2 = hd.Operator.from_workload(w2)
        f32 = phi[:nl]
        phi64 = f32.to(torch.complex128)
        bf = torch.view_as_real(f32).to(torch.bfloat16).contiguous()
        ref = hd.born_apply(op2, phi64[:, :S], phi64[:, S:], vv.double())
        cases = [("fp32", f32, False, FP32_PEAK_TFLOPS, 8), ("split_bf16", f32, True, BF16_PEAK_TFLOPS, 8),
                 ("bf16_fields", bf, False, BF16_PEAK_TFLOPS, 4)]
        for name, f, split, peak, bpc in cases:
            ms = timed(lambda: hd.born_apply(op2, f[:, :S], f[:, S:], vv, split_bf16=split))
            y = hd.born_apply(op2, f[:, :S], f[:, S:], vv, split_bf16=split)
            n_v = vv.shape[0]
            L2 = nl
            useful = 8.0 * S * D * N * L2 * n_v
            pairs = n_v >= hd.BORN_PAIRS_MIN_NV
            # MFMA work the kernel executes: the real-ified complex product (8 S D N per probe vector,
            # rows padded to 8), or with the pair-product kernel 4 S D N per probe vector, pairs in
            # tiles of 8 x 8 and probe vectors padded to a multiple of 16; split-BF16: three products
            executed = (4.0 * pad(S, 8) * pad(D, 8) * N * L2 * pad(n_v, 16) if pairs
                        else 8.0 * pad(S, 8) * pad(D, 8) * N * L2 * n_v) * (3 if split else 1)
            needed = (4.0 * S * D * N * L2 * n_v if pairs else useful) * (3 if split else 1)
            err = float(torch.linalg.vector_norm(y.to(torch.complex128) - ref) / torch.linalg.vector_norm(ref))
            out[f"{name}_nv{nv}"] = {
                "kernel": ("k_born_jv_pairs" if pairs else "k_born_jv" if S <= 32 or D <= 32
                           else "k_born_jv_wide" if name == "fp32" else "k_born_jv_wide_bf"),
                "wavelengths": nl, "ms": round(ms, 4),
                "tflops_8SDNL_convention": round(useful / (ms * 1e-3) / 1e12, 2),
                "mfma_tflops_needed": round(needed / (ms * 1e-3) / 1e12, 2),
                "mfma_frac_needed": round(needed / (ms * 1e-3) / 1e12 / peak, 4),
                "mfma_tflops_executed_padded": round(executed / (ms * 1e-3) / 1e12, 2),
                "mfma_frac_executed_padded": round(executed / (ms * 1e-3) / 1e12 / peak, 4), "mfma_peak_tflops": peak,
                "field_GBps": round((S + D) * N * L2 * bpc / (ms * 1e-3) / 1e9, 1),
                "rel_err_vs_fp64_products": float(f"{err:.3g}")}
        if nv == "1":
            # J^H w from BF16-stored fields (BF16 MFMA, w split into hi + lo) beside the FP32 one
            wv = torch.from_numpy(workloads.born_w(w)[:nl]).to(torch.complex64).to(dev)
            gref = hd.born_apply_adjoint(op2, phi64[:, :S], phi64[:, S:], wv.to(torch.complex128))
            for name, f, bpc in (("fp32", f32, 8), ("bf16_fields", bf, 4)):
                ms = timed(lambda: hd.born_apply_adjoint(op2, f[:, :S], f[:, S:], wv))
                gg = hd.born_apply_adjoint(op2, f[:, :S], f[:, S:], wv)
                err = float(torch.linalg.vector_norm(gg.to(torch.complex128) - gref) / torch.linalg.vector_norm(gref))
                flops = 8.0 * S * D * N * nl
                peak = FP32_PEAK_TFLOPS if name == "fp32" else BF16_PEAK_TFLOPS
                out[f"adjoint_{name}"] = {
                    "kernel": "k_born_adjoint_wide" if name == "fp32" else "k_born_adjoint_wide_bf",
                    "wavelengths": nl, "ms": round(ms, 4),
                    "tflops_8SDNL_convention": round(flops / (ms * 1e-3) / 1e12, 2),
                    "mfma_frac_executed": round(flops * (1 if name == "fp32" else 2) / (ms * 1e-3) / 1e12 / peak, 4),
                    "mfma_peak_tflops": peak,
                    "field_GBps": round((S + D) * N * nl * bpc / (ms * 1e-3) / 1e9, 1),
                    "hbm_frac": round((S + D) * N * nl * bpc / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "rel_err_vs_fp64_products": float(f"{err:.3g}")}
            del gref
        del phi64, bf
    out["note"] = ("shard 0: one probe vector on all its wavelengths, the 42-vector block on two, J^H w of one data "
                   "vector on all its wavelengths (BF16 fields: w split into two BF16 products); 'needed' counts "
                   "the multiply-adds the algorithm needs (4 S D N per "
                   "probe vector on the pair-product kernel, whose pair products are shared by the probe vectors; "
                   "8 S D N on the real-ified kernel), 'executed_padded' includes the padding of rows to 8 and of "
                   "probe vectors to 16, and the 8*S*D*N*L convention credits every probe vector with a full complex "
                   "product (it can exceed the MFMA peak on the pair-product kernel)")
    return out


def run_studies(hd, torch, np, workloads, w, op, opts, phi, dev, p_true, dc_true):
    """Secondary measurements on one shard (not part of the step): heterogeneous forward with the PaLS
    anomaly and the Born validity, boundary split and shift variants, the separable preconditioner."""
    S, R, L = w.S, w.S + w.D, w.L
    vox = w.rhs_voxels
    out = {}
    det = torch.from_numpy(np.asarray(w.det_voxels)).to(dev)
    hd.solve_fields(op, vox, opts, out=phi)
    d0 = phi[:, :S][:, :, det].to(torch.complex128)
    shape_t = hd.pals_shape(op, p_true, device=dev)
    Jmu64 = hd.born_apply(op, phi[:, :S].to(torch.complex128), phi[:, S:].to(torch.complex128), shape_t[None])[0]
    ebar_true = dc_true @ w.extinction
    op.set_absorption_perturbation(shape_t.cpu().numpy(), ebar_true)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    _, fit, frel, _ = hd.solve_fields(op, vox, opts, out=phi)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    dfull = phi[:, :S][:, :, det].to(torch.complex128) - d0
    pred = torch.from_numpy(ebar_true).to(dev)[:, None, None] * Jmu64
    mism = float(torch.linalg.vector_norm(dfull - pred) / torch.linalg.vector_norm(dfull))
    op.set_absorption_perturbation(None, None)
    out["forward_heterogeneous"] = {"solves_per_s": round(R * L / (tb - ta), 1), "max_rel_res": float(frel.max()),
                                    "mean_iters": float(fit.mean()),
                                    "born_relative_mismatch_at_detectors": float(f"{mism:.3g}")}
    log("heterogeneous forward done")
    study = {}
    wb = workloads.Workload(**{**w.__dict__, "robin_faces": 0x30})
    opb = hd.Operator.from_workload(wb)
    for bname, bop, shifts in (("all_robin", op, ("mean",)), ("robin_top_bottom", opb, ("mean", "min", "max", "none"))):
        for sname in shifts:
            fl = {"mean": hd.FLAG_MEAN_SHIFT, "min": hd.FLAG_SHIFT_MIN, "max": hd.FLAG_SHIFT_MAX, "none": 0}[sname]
            so = hd.SolveOptions(**{**opts.__dict__, "flags": fl | hd.FLAG_GRAPH})
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, sit, srel, _ = hd.solve_fields(bop, vox, so, out=phi)
            torch.cuda.synchronize()
            study[f"{bname}/{sname}"] = {"solves_per_s": round(R * L / (time.perf_counter() - ta), 1),
                                         "mean_iters": round(float(sit.mean()), 2), "max_rel_res": float(srel.max())}
    out["boundary_shift"] = study
    log("boundary/shift study done")
    pstudy = {}
    for pname, pfl in (("none", 0), ("sep", hd.FLAG_PRECOND_SEP), ("sep_fixed", hd.FLAG_PRECOND_SEP_FIXED)):
        so = hd.SolveOptions(**{**opts.__dict__, "flags": hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH | pfl})
        torch.cuda.synchronize()
        ta = time.perf_counter()
        _, sit, srel, _ = hd.solve_fields(op, vox, so, out=phi)
        torch.cuda.synchronize()
        pstudy[pname] = {"solves_per_s": round(R * L / (time.perf_counter() - ta), 1),
                         "mean_iters": round(float(sit.mean()), 2), "max_rel_res": float(srel.max())}
    out["preconditioner"] = pstudy
    log("preconditioner study done")
    return out


if __name__ == "__main__":
    main()
