#!/usr/bin/env python3
"""Throughput of the hyperspectral DOT Born hot path on one MI355X.

One step = the whole hot path over one synthetic workload:
  fields for every source and detector at every wavelength (Algorithm 1 with a
  recycled deflation space, all systems batched, complex FP32 Krylov with FP64
  residual refinement to rel-res 1e-8) -> Born J v -> Born J^H w -> PaLS misfit
  value and gradient (forward + adjoint).

Prints one JSON line.  value = RHS x wavelength solves per second of whole steps.
Extra fields: Born J v GFLOP/s, the plain per-system FP64 solver's rate on a
subsample (one right-hand side, every wavelength), the roofline of the dominant
kernel (HIP events inside the library, on the solve stream), and the CPU oracle
timed on a bounded sample.
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

# Solver settings of the batched path: deflation space k = 5, m - k = 13 Arnoldi steps per
# cycle, 32 shift-invariant Lanczos steps (the fastest setting of a sweep over k, m, n and the
# inner tolerance on the medium workload).
RECYCLE_K, RESTART_M, LANCZOS_N = 5, 18, 32

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0   # dense MFMA
N_JAC = 42                  # Jacobian block: 2 chromophore contrasts + 40 PaLS parameters

# Calibrated HBM bytes per dispatch of the Arnoldi step kernels on the medium workload,
# from the FETCH_SIZE / WRITE_SIZE runs summarised in profiles/step_kernels_medium_traffic.md.
# They belong to the kernel sources with this SHA-256 (common.h, krylov_kernels.h,
# krylov_tiled.h); after any change to those the traffic is reported as null.
# They also hold only for the launch shape they were taken with (TRAFFIC_TUNING), per block order.
TRAFFIC_SOURCES_SHA256 = "db11902b439aa098e59265b181e4e63e2e154095c35ef4fa49d6b36b052d0287"
TRAFFIC_TUNING = {"step_presum": 16, "step_group": 2, "step_vx": 1}
TRAFFIC_BYTES_PER_LAUNCH = {   # step_order -> kernel -> calibrated HBM bytes per launch
    3: {"k_step_dots_t": 5.320e9, "k_step_update_t": 6.051e9, "k_step_finish_t": 1.208e6},
    2: {"k_step_dots_t": 6.229e9, "k_step_update_t": 6.982e9, "k_step_finish_t": 1.208e6},
}


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("common.h", "krylov_kernels.h", "krylov_tiled.h"):
        with open(os.path.join(ROOT, "paper_1410_0986_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()

WORKLOAD_TEXT = {
    "medium": "medium: 64x64x32 grid (131072 voxels, h=2 mm), 16 sources + 16 detectors, 32 wavelengths 650-900 nm",
    "batch": "batch: 64x64x32 grid (131072 voxels, h=2 mm), 32 sources + 32 detectors, 64 wavelengths 650-900 nm",
    "tiny": "tiny: 16x16x8 grid (2048 voxels, h=2 mm), 4 sources + 4 detectors, 8 wavelengths 650-860 nm",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(wname: str, n_sys: int):
    """Unrecycled GMRES(30) of the FP64 oracle on a bounded sample of the same workload."""
    import numpy as np
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
            "sample": f"{len(lams)} systems (source 0 at wavelengths {lams}) of the {wname} workload, "
                      f"unrecycled GMRES(30) FP64 to 1e-8, {iters} iterations, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="medium", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-system FP64 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default="",
                    help="launch-shape fields set after the autotuner, e.g. step_order=3,step_group=2")
    ap.add_argument("--no-studies", action="store_true",
                    help="skip the secondary measurements after the Born variants (heterogeneous forward, "
                         "boundary/shift study, compression, reconstruction), e.g. under a profiler")
    ap.add_argument("--born-only", action="store_true",
                    help="only the Born J v variants (one solve for the fields, no autotuner, no timed steps)")
    ap.add_argument("--cpu-sample", type=int, default=10, help="systems in the CPU oracle sample")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="finish with one device-to-device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the hot path is measured on one GPU's share; see the sharding notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1410_0986_amd as hd
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)     # default priority
    w = workloads.config(args.config)
    op = hd.Operator.from_workload(w)
    S, D, L, N = w.S, w.D, w.L, w.N
    R = S + D
    vox = w.rhs_voxels
    opts = hd.SolveOptions(rel_tol=1e-8, restart_m=RESTART_M, recycle_k=RECYCLE_K, lanczos_n=LANCZOS_N,
                           precision=hd.PREC_MIXED, inner_tol=1e-5, flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH,
                           max_iter=5000)
    v = torch.from_numpy(workloads.born_v(w, dtype=np.float32)).to(dev)
    wv = torch.from_numpy(workloads.born_w(w)).to(torch.complex64).to(dev)
    p_true, dc_true = workloads.pals_truth(w)
    p_eval, dc_eval = workloads.pals_perturbed(w, p_true, dc_true)

    with torch.cuda.stream(stream):
        phi = torch.empty((L, R, N), dtype=torch.complex64, device=dev)

        def solve():
            return hd.solve_fields(op, vox, opts, out=phi)

        def born_variants():
            # Born variants (not part of the step): FP32 / BF16-stored / split-BF16 products for one
            # probe vector and for the Jacobian block, each against the FP64 products of the same fields
            phi_bf = torch.empty((L, R, N, 2), dtype=torch.bfloat16, device=dev)
            hd.solve_fields(op, vox, opts, out=phi_bf)
            phi64 = phi.to(torch.complex128)
            vj = torch.from_numpy(workloads.born_v(w, n_v=N_JAC, seed=2024, dtype=np.float32)).to(dev)

            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

            def timed(fn, nrep=10):
                fn()
                e0.record(stream)
                for _ in range(nrep):
                    fn()
                e1.record(stream)
                e1.synchronize()
                return e0.elapsed_time(e1) / nrep

            variants = {}
            for nv, vv in (("1", v), (str(N_JAC), vj)):
                ref = hd.born_apply(op, phi64[:, :S], phi64[:, S:], vv.double())
                cases = [("fp32", phi, False, FP32_PEAK_TFLOPS, 8), ("split_bf16", phi, True, BF16_PEAK_TFLOPS, 8),
                         ("bf16_fields", phi_bf, False, BF16_PEAK_TFLOPS, 4)]
                for name, f, split, peak, bpc in cases:
                    ms = timed(lambda: hd.born_apply(op, f[:, :S], f[:, S:], vv, split_bf16=split))
                    y = hd.born_apply(op, f[:, :S], f[:, S:], vv, split_bf16=split)
                    n_v = vv.shape[0]
                    fl = 8.0 * S * D * N * L * n_v
                    # MFMA work the kernel executes: the real-ified complex product (8 S D N per probe
                    # vector, rows padded to 8), or with the pair-product kernel (hd.BORN_PAIRS_MIN_NV
                    # or more probe vectors) 4 S D N per probe vector, pairs in tiles of 8 x 8 and
                    # probe vectors padded to a multiple of 16; split-BF16 runs three BF16 products
                    pairs = n_v >= hd.BORN_PAIRS_MIN_NV
                    pad = lambda x, m: -(-x // m) * m
                    fl_mfma = (4.0 * pad(S, 8) * pad(D, 8) * N * L * pad(n_v, 16) if pairs
                               else 8.0 * pad(S, 8) * pad(D, 8) * N * L * n_v) * (3 if split else 1)
                    err = float(torch.linalg.vector_norm(y.to(torch.complex128) - ref) / torch.linalg.vector_norm(ref))
                    variants[f"{name}_nv{nv}"] = {
                        "kernel": "k_born_jv_pairs" if pairs else "k_born_jv",
                        "ms": round(ms, 4), "tflops": round(fl / (ms * 1e-3) / 1e12, 2),
                        "mfma_tflops_executed": round(fl_mfma / (ms * 1e-3) / 1e12, 2),
                        "mfma_frac": round(fl_mfma / (ms * 1e-3) / 1e12 / peak, 4), "mfma_peak_tflops": peak,
                        "field_GBps": round((S + D) * N * L * bpc / (ms * 1e-3) / 1e9, 1),
                        "rel_err_vs_fp64_products": float(f"{err:.3g}")}
            del phi_bf, phi64
            return variants

        if args.born_only:
            # the Born variants alone on the fields of one solve (default launch shapes), e.g. under
            # a counter profiler
            solve()
            print(json.dumps({"born_variants": born_variants()}), flush=True)
            return

        # launch shapes: the autotuner times its candidates on this problem (set-up, not timed)
        solve_trials = hd.autotune_solve(op, vox, opts, out=phi)
        log(f"autotune of the step kernels done ({len(solve_trials)} candidates)")
        for t, ms in solve_trials:
            log(f"  presum {t['step_presum']} vx {t['step_vx']} order {t['step_order']} group {t['step_group']}: "
                f"{ms:.1f} ms")
        if args.tuning:
            hd.set_tuning(op, **{k: int(x) for k, x in (kv.split("=") for kv in args.tuning.split(","))})
            log(f"tuning set to {hd.get_tuning(op)}")
        # observed data of the PaLS model at the truth (set-up, not timed)
        solve()
        born_trials = hd.autotune_born(op, phi[:, :S], phi[:, S:], v)
        log(f"autotune of J v done ({len(born_trials)} candidates)")
        for t, ms in born_trials:
            log(f"  stage {t['born_stage']} blocks {t['born_blocks']}: {ms:.4f} ms")
        mu_t = hd.pals_shape(op, p_true, dtype=torch.float32, device=dev)
        Jmu = hd.born_apply(op, phi[:, :S], phi[:, S:], mu_t[None])[0]
        ebar = torch.from_numpy(dc_true @ w.extinction).to(dev).to(torch.float32)
        y_obs = (ebar[:, None, None] * Jmu).contiguous()

        def step():
            _, it, rel, st = solve()
            y = hd.born_apply(op, phi[:, :S], phi[:, S:], v)
            g = hd.born_apply_adjoint(op, phi[:, :S], phi[:, S:], wv)
            dct = torch.tensor(dc_eval, requires_grad=True)
            pt = torch.tensor(p_eval, requires_grad=True)
            f = hd.BornMisfit.apply(dct, pt, op, phi[:, :S], phi[:, S:], y_obs)
            f.backward()
            return it, rel, st, y, g

        for i in range(args.warmup):
            step()
            log(f"warmup step {i + 1}/{args.warmup} done")
        torch.cuda.synchronize()
        hd.profile_enable(True)
        t0 = time.perf_counter()
        its, rels = [], []
        for i in range(args.steps):
            it, rel, st, _, _ = step()
            its.append(it)
            rels.append(rel)
            log(f"timed step {i + 1}/{args.steps} done")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = hd.profile_read()
        hd.profile_enable(False)

        # Born J v alone (GFLOP/s) and J^H w alone, HIP events on this stream
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        hd.born_apply(op, phi[:, :S], phi[:, S:], v)
        e0.record(stream)
        for _ in range(reps):
            hd.born_apply(op, phi[:, :S], phi[:, S:], v)
        e1.record(stream)
        e1.synchronize()
        jv_ms = e0.elapsed_time(e1) / reps
        e0.record(stream)
        for _ in range(reps):
            hd.born_apply_adjoint(op, phi[:, :S], phi[:, S:], wv)
        e1.record(stream)
        e1.synchronize()
        jhw_ms = e0.elapsed_time(e1) / reps
        log("born timing done")

        variants = born_variants()
        log("born variants done")

        forward = study = compression = reconstruction = None
        if not args.no_studies:
            # full forward model with the PaLS anomaly at the true contrast (not part of the step):
            # throughput of the recycled solver on the heterogeneous operator, and the Born validity
            # (relative mismatch of the detector-data change against the Born prediction)
            det = torch.from_numpy(np.asarray(w.det_voxels)).to(dev)
            d0 = phi[:, :S][:, :, det].to(torch.complex128)
            shape_t = hd.pals_shape(op, p_true, device=dev)
            Jmu64 = hd.born_apply(op, phi[:, :S].to(torch.complex128), phi[:, S:].to(torch.complex128),
                                  shape_t[None])[0]
            ebar_true = dc_true @ w.extinction
            op.set_absorption_perturbation(shape_t.cpu().numpy(), ebar_true)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, fit, frel, fst = hd.solve_fields(op, vox, opts, out=phi)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            dfull = phi[:, :S][:, :, det].to(torch.complex128) - d0
            pred = torch.from_numpy(ebar_true).to(dev)[:, None, None] * Jmu64
            born_mismatch = float(torch.linalg.vector_norm(dfull - pred) / torch.linalg.vector_norm(dfull))
            op.set_absorption_perturbation(None, None)

            forward = {"solves_per_s": round(R * L / (tb - ta), 1), "max_rel_res": float(frel.max()),
                       "mean_iters": float(fit.mean()),
                       "born_relative_mismatch_at_detectors": float(f"{born_mismatch:.3g}"),
                       "anomaly": "PaLS truth (8 bumps), contrast dc = (8, 8) uM"}
            log("heterogeneous forward done")

            # boundary split and shift-variant study (Sec. 6.1 setting): the paper's plates (Robin on
            # the top and bottom faces, Dirichlet on the sides) with sigma' moved into K_hat as its mean,
            # minimum, maximum or not at all, against the all-Robin box with the mean shift
            study = {}
            wb = workloads.config(args.config, robin_faces=0x30)
            opb = hd.Operator.from_workload(wb)
            for bname, bop, shifts in (("all_robin", op, ("mean",)), ("robin_top_bottom", opb, ("mean", "min", "max", "none"))):
                for sname in shifts:
                    fl = {"mean": hd.FLAG_MEAN_SHIFT, "min": hd.FLAG_SHIFT_MIN, "max": hd.FLAG_SHIFT_MAX,
                          "none": 0}[sname] | hd.FLAG_GRAPH
                    so = hd.SolveOptions(rel_tol=1e-8, restart_m=RESTART_M, recycle_k=RECYCLE_K, lanczos_n=LANCZOS_N,
                                         precision=hd.PREC_MIXED, inner_tol=1e-5, flags=fl, max_iter=5000)
                    torch.cuda.synchronize()
                    ta = time.perf_counter()
                    _, sit, srel, sst = hd.solve_fields(bop, vox, so, out=phi)
                    torch.cuda.synchronize()
                    tb = time.perf_counter()
                    study[f"{bname}/{sname}"] = {"solves_per_s": round(R * L / (tb - ta), 1),
                                                 "mean_iters": round(float(sit.mean()), 2),
                                                 "max_rel_res": float(srel.max())}
            del opb
            log("boundary/shift study done")

            # preconditioner study (Sec. 6.1 preconditions with an ILU of the mean-shifted matrix):
            # the separable preconditioner with each system's own shift or one shift for all, on the
            # homogeneous box and with the PaLS anomaly, against no preconditioner
            pstudy = {}
            for aname, anom in (("homogeneous", False), ("pals_anomaly", True)):
                if anom:
                    op.set_absorption_perturbation(shape_t.cpu().numpy(), ebar_true)
                for pname, pfl in (("none", 0), ("sep", hd.FLAG_PRECOND_SEP), ("sep_fixed", hd.FLAG_PRECOND_SEP_FIXED)):
                    so = hd.SolveOptions(rel_tol=1e-8, restart_m=RESTART_M, recycle_k=RECYCLE_K, lanczos_n=LANCZOS_N,
                                         precision=hd.PREC_MIXED, inner_tol=1e-5,
                                         flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_GRAPH | pfl, max_iter=5000)
                    torch.cuda.synchronize()
                    ta = time.perf_counter()
                    _, sit, srel, sst = hd.solve_fields(op, vox, so, out=phi)
                    torch.cuda.synchronize()
                    tb = time.perf_counter()
                    pstudy[f"{aname}/{pname}"] = {"solves_per_s": round(R * L / (tb - ta), 1),
                                                  "mean_iters": round(float(sit.mean()), 2),
                                                  "max_rel_res": float(srel.max())}
                if anom:
                    op.set_absorption_perturbation(None, None)
            study["preconditioner"] = pstudy
            log("preconditioner study done")

            # randomized compression of H (Sec. 4): recursive over the source bisection tree against one
            # randomized SVD of the whole H, tolerance 1e-3, error measured with fresh probe vectors
            from paper_1410_0986_amd import compress as hcompress
            hd.solve_fields(op, vox, opts, out=phi)
            xy = workloads.optode_xy(w, w.src_voxels)
            om1 = workloads.gaussian_test_matrix(N, 700)
            om2 = workloads.gaussian_test_matrix(N, 10, seed=workloads.COMPRESS_SEED + 1)
            vprobe = torch.from_numpy(workloads.born_v(w, n_v=8, seed=99, dtype=np.float32)).to(dev)
            yprobe = hd.born_apply(op, phi[:, :S], phi[:, S:], vprobe).permute(0, 2, 1, 3).reshape(8, -1)
            yprobe = yprobe.to(torch.complex128)
            cb = hcompress.compress(op, phi[:, :S], phi[:, S:], xy, 1e-3, om1[:, :300], om2)
            cerr = float(torch.linalg.vector_norm(cb.matvec(vprobe) - yprobe) / torch.linalg.vector_norm(yprobe))
            torch.cuda.synchronize()
            td = time.perf_counter()
            lr = hcompress.randsvd_direct(op, phi[:, :S], phi[:, S:], 1e-3, om1, om2)
            torch.cuda.synchronize()
            tdir = time.perf_counter() - td
            dy = (lr.U @ (lr.V.conj().T @ vprobe.to(torch.complex128).T)).T
            derr = float(torch.linalg.vector_norm(dy - yprobe) / torch.linalg.vector_norm(yprobe))
            compression = {"eps": 1e-3, "rows": S * L * D, "cols": N,
                           "recursive": {"seconds": round(cb.seconds, 3), "rank": cb.rank,
                                         "rank_before_recompression": cb.recursive_rank,
                                         "level_ranks": {str(k): v for k, v in sorted(cb.level_ranks.items())},
                                         "probe_rel_err": float(f"{cerr:.3g}"), "H_columns_applied": cb.products},
                           "direct_randsvd": {"seconds": round(tdir, 3), "rank": lr.rank,
                                              "probe_rel_err": float(f"{derr:.3g}"), "H_columns_applied": lr.products}}
            del lr
            log("compression done")

            # reconstruction (Sec. 5, Alg. opt) on these fields: Exp. 1 analogue (3 bumps, known
            # contrasts, 33 dB, full H against H compressed at 1e-3 and 1e-6) and Exp. 2 analogue
            # (contrasts too, 30 dB, random start, H compressed at 1e-6); data from the full H
            from paper_1410_0986_amd import reconstruct as hrec
            cbs = {1e-3: cb, 1e-6: hcompress.compress(op, phi[:, :S], phi[:, S:], xy, 1e-6, om1, om2)}
            log("compression at 1e-6 done")
            del om1
            p3, _ = workloads.pals_truth(w, n_bumps=3)
            mu3 = hd.pals_shape(op, p3, dtype=torch.float32, device=dev)
            full_model = hrec.BornModel(op, phi[:, :S], phi[:, S:], w.extinction)
            y_clean = (dc_true @ w.extinction)[:, None, None] * full_model.H(mu3[None])[0]
            mu3_np = mu3.double().cpu().numpy()

            def recon(model, snr_db, p0, fix_c):
                eta = workloads.observed_noise(y_clean.shape, 10 ** (-snr_db / 20) * np.linalg.norm(y_clean)
                                               / np.sqrt(y_clean.size), seed=34 + int(snr_db))
                r = hrec.reconstruct(model, y_clean + eta, p0, c0=dc_true if fix_c else None,
                                     noise_norm=float(np.linalg.norm(eta)), fix_c=fix_c, max_outer=300)
                mu_r = hd.pals_shape(op, r.p, device=dev).cpu().numpy()
                l2, dice = hrec.shape_errors(mu3_np, mu_r)
                return {"L2_err": round(l2, 4), "dice": round(dice, 3), "seconds": round(r.seconds, 3),
                        "outer": r.outer, "lm_steps": r.lm_steps, "stopped_by": r.stopped_by,
                        "conc_rel_err": [round(abs(a - b) / abs(b), 4) for a, b in zip(r.c, dc_true)]}

            p_start, _ = workloads.pals_perturbed(w, p3, dc_true)
            exp1 = {"full_H": recon(full_model, 33.0, p_start, True)}
            log("reconstruction with the full H done")
            for e_, cbe in cbs.items():
                mdl = hrec.BornModel(op, phi[:, :S], phi[:, S:], w.extinction, compressed=cbe)
                exp1[f"{e_:g}"] = {"rank": cbe.rank, "compress_seconds": round(cbe.seconds, 3),
                                   **recon(mdl, 33.0, p_start, True)}
                log(f"reconstruction with H compressed at {e_:g} done")
            mdl6 = hrec.BornModel(op, phi[:, :S], phi[:, S:], w.extinction, compressed=cbs[1e-6])
            exp2 = recon(mdl6, 30.0, workloads.pals_random_start(w, 3), False)
            reconstruction = {"measurements": S * D * L, "n_p": 15, "exp1_shape_only_33dB": exp1,
                              "exp2_shape_and_conc_30dB_random_start_eps1e-6": exp2}
            del cb, cbs, mdl6
            log("reconstruction done")


        plain = None
        if not args.no_plain:
            w1 = workloads.Workload(**{**w.__dict__, "src_voxels": w.src_voxels[:1],
                                       "det_voxels": w.det_voxels[:0], "extra": {}})
            op1 = hd.Operator.from_workload(w1)
            po = hd.SolveOptions(rel_tol=1e-8, restart_m=RESTART_M, recycle_k=RECYCLE_K, lanczos_n=LANCZOS_N,
                                 precision=hd.PREC_FP64,
                                 flags=hd.FLAG_MEAN_SHIFT | hd.FLAG_PER_SYSTEM, max_iter=5000)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, pit, prel, pst = hd.solve_fields(op1, w1.rhs_voxels, po, device=dev)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            plain = {"solves_per_s": L / (tb - ta), "sample": f"1 right-hand side x {L} wavelengths",
                     "max_rel_res": float(prel.max()), "mean_iters": float(pit.mean())}
            log("plain path done")

    if args.copy_gib > 0:
        nbytes = int(args.copy_gib * (1 << 30))
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy of {nbytes} bytes done")
        del a, b

    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / args.steps
    solves_per_s = R * L * args.steps / elapsed
    rel_all = np.stack(rels)
    it_all = np.stack(its)
    jv_flops = 8.0 * S * D * N * L
    # dominant kernel by time
    name, (launches, kms, kbytes) = max(prof.items(), key=lambda kv: kv[1][1])
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    traffic = None
    tuned = hd.get_tuning(op)
    if args.config == "medium" and kernel_sources_sha256() == TRAFFIC_SOURCES_SHA256 and \
            all(tuned[k] == v for k, v in TRAFFIC_TUNING.items()):
        traffic = TRAFFIC_BYTES_PER_LAUNCH.get(tuned["step_order"], {}).get(name)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "bytes/launch",
            "kernel": name,
            "launches": launches, "avg_launch_ms": round(kms / max(launches, 1), 4),
            "algorithmic_bytes_per_launch": kbytes / max(launches, 1),
            "all_step_kernels": {k: {"launches": a, "ms": round(b, 2), "GB/s": round(c / (b * 1e-3) / 1e9, 1)
                                     if b > 0 else 0.0} for k, (a, b, c) in prof.items()}}
    out = {
        "metric": "RHS x wavelength solves/sec at rel-res 1e-8 (+ Born Jv GFLOP/s), batched vs plain",
        "value": round(solves_per_s, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 Krylov + f64 refinement",
        "data": "synthetic (seeded)",
        "config": {"workload": WORKLOAD_TEXT[args.config], "systems_per_step": R * L,
                   "solver": f"batched recycled GMRES, m={RESTART_M}, k={RECYCLE_K}, n={LANCZOS_N}, mean shift, "
                             "FP32 inner to 1e-5",
                   "max_rel_res": float(rel_all.max()), "mean_iters": float(it_all.mean())},
        "born_jv_gflops": round(jv_flops / (jv_ms * 1e-3) / 1e9, 1),
        "born_jv_ms": round(jv_ms, 4),
        "born_jv_mfma_frac_fp32": round(jv_flops / (jv_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
        "born_adjoint_ms": round(jhw_ms, 4),
        # the MFMA-bound Born configuration: FP32 J v of the 42-column PaLS Jacobian block
        "born_jv_jacobian_block": {k: variants[f"fp32_nv{N_JAC}"][k] for k in
                                   ("kernel", "ms", "tflops", "mfma_tflops_executed", "mfma_frac",
                                    "rel_err_vs_fp64_products")},
        "born_variants": variants,
        "forward_heterogeneous": forward,
        "boundary_shift_study": study,
        "compression": compression,
        "reconstruction": reconstruction,
        "plain_fp64": plain,
        "speedup_vs_plain": round(solves_per_s / plain["solves_per_s"], 2) if plain else None,
        "roofline": roof,
        "tuning": {**hd.get_tuning(op), "solve_candidates": len(solve_trials),
                   "born_candidates": len(born_trials)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.config, args.cpu_sample)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
