#!/usr/bin/env python
"""Interaction-matrix build benchmark on one MI355X.

Workload: the ELT-scale SCAO IM in FP32 - 80x80 subapertures of 6 px on a
480-px pupil with 28% central obscuration (4632 valid subapertures), a 81x81
Gaussian-IF DM (5257 actuators inside the pupil, 512^2 IF grid, 5.5 GB stack
resident in HBM) and a seeded misregistration.  One step = one full IM build
(geometry plan + streaming pass over every IF) = 5257 IM columns.

Printed JSON line: IM columns/s of the whole step, the streaming kernel's
achieved algorithmic HBM bandwidth against the 8 TB/s peak (HIP events on the
launch stream), and the FP64 oracle's rate on a bounded sample of the same
workload on the host cores.

    python bench.py [--steps K] [--warmup W] [--seed S] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IM columns/s & % HBM roofline; misreg-fit ms, learned vs Gauss-Newton"
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "im_stream_elt_traffic.json")
MCAO_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "im_stream_mcao_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------ algorithmic bytes
def touched_mask(pupil, p: int, valid, A, grid_n: int):
    """Boolean [grid_n][grid_n] mask of the IF pixels with a non-zero bilinear
    weight for some sample that the central differences read (the
    4-neighbours of every pupil pixel of a valid subaperture).  Depends on the
    geometry only, not on any kernel."""
    import numpy as np
    H, W = pupil.shape
    ns = W // p
    use = np.zeros((H, W), bool)
    for k in valid:
        v, u = divmod(int(k), ns)
        use[v * p:(v + 1) * p, u * p:(u + 1) * p] = pupil[v * p:(v + 1) * p, u * p:(u + 1) * p] > 0
    Q = np.zeros((H + 2, W + 2), bool)          # haloed sample grid
    Q[1:-1, 2:] |= use
    Q[1:-1, :-2] |= use
    Q[2:, 1:-1] |= use
    Q[:-2, 1:-1] |= use
    yy, xx = np.nonzero(Q)
    x = xx - 1.0
    y = yy - 1.0
    xs = A[0, 0] * x + A[0, 1] * y + A[0, 2]
    ys = A[1, 0] * x + A[1, 1] * y + A[1, 2]
    i = np.floor(xs).astype(np.int64)
    j = np.floor(ys).astype(np.int64)
    a = xs - i
    c = ys - j
    S = np.zeros((grid_n, grid_n), bool)
    for di, dj, w in ((0, 0, (1 - a) * (1 - c)), (1, 0, a * (1 - c)), (0, 1, (1 - a) * c), (1, 1, a * c)):
        nz = w != 0
        ii = i[nz] + di
        jj = j[nz] + dj
        ok = (ii >= 0) & (ii < grid_n) & (jj >= 0) & (jj < grid_n)
        S[jj[ok], ii[ok]] = True
    return S


def touched_if_pixels(cfg, A) -> int:
    """|S| of one SCAO workload (see touched_mask)."""
    return int(touched_mask(cfg.pupil, cfg.p, cfg.valid, A, cfg.grid.grid_n).sum())


# ----------------------------------------------------------------- CPU baseline
def _oracle_chunk(args):
    seed, cols = args
    import numpy as np
    import workloads as wl
    from oracle import geometry as og, im as oim
    cfg = wl.scao_elt(seed)
    A, b = og.inverse_from_misreg(cfg.theta, 512, 512, cfg.n_out, cfg.n_out)
    F = np.stack([wl.if_single(cfg.grid, a) for a in cols])
    t0 = time.perf_counter()
    oim.im_build(F, A, b, cfg.pupil, cfg.p, cfg.valid)
    return time.perf_counter() - t0


def cpu_baseline(seed: int, target_s: float):
    """FP64 oracle on a bounded sample of the same workload, on the host cores.

    Runs before the GPU is touched, in a pool of spawned worker processes."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import numpy as np
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    # one GPU's share of the host is 16 CPUs on the GPU machines: more worker
    # processes than that would take cores the GPU's own host work needs
    workers = max(1, min(16, ncpu))
    chunk = 4
    # calibrate on one chunk in-process: the one-core rate
    t1 = _oracle_chunk((seed, list(range(chunk))))
    per_col = t1 / chunk
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n_cols = int(max(workers * chunk, min(5257, target_s * workers / per_col)))
    n_cols = min(5256, (n_cols + chunk - 1) // chunk * chunk)
    cols = np.linspace(0, 5256, n_cols).astype(int).tolist()
    jobs = [(seed, cols[i:i + chunk]) for i in range(0, n_cols, chunk)]
    log(f"cpu baseline: {n_cols} columns on {workers} workers (~{per_col:.3f} s/column/core)")
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        list(ex.map(_oracle_chunk, jobs))
    wall = time.perf_counter() - t0
    return {"value": n_cols / wall, "unit": "IM columns/s", "cores": workers, "kind": "oracle",
            "sample": f"{n_cols} of 5257 IM columns of the ELT workload (seed {seed}), FP64 "
                      f"NumPy oracle, {workers} worker processes, {wall:.1f} s wall",
            "one_core_value": 1.0 / per_col, "cpu_model": cpu_model,
            "host_cpus": os.cpu_count(), "affinity_cpus": ncpu,
            "workers_note": "worker processes capped at 16, one GPU's share of the host CPUs"}


def stored_traffic(record=TRAFFIC_FILE):
    """HBM bytes per launch of a streaming kernel (rocprofv3 FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy's counts) from a committed counter
    record, if it was taken on the current source of the files it names (the
    stream kernel and the plan that builds its tiles); else None."""
    try:
        with open(record) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if rec.get("kernel_sha") != h.hexdigest()[:16]:
            return None
        return float(rec["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


# ------------------------------------------------------------- further legs
def _event_ms(fn, reps: int):
    """Mean ms of fn() over reps, HIP events on torch's current stream (every
    launch of fn is ordered on it)."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def mcao_leg(synim, dev, reps: int = 10):
    """Multi-WFS batch: 6 LGS WFS x 3 DMs (18 pair maps), one persistent
    launch per patch size (the 15-deg and 45-deg clocked WFS need different
    patches), replayed as a hipGraph.  Algorithmic bytes: each DM's IF pixels
    touched by the union of its 6 WFS footprints, read once, plus every
    pair's IM."""
    import numpy as np
    import torch
    import workloads as wl
    cfg = wl.mcao(0)
    stacks = [wl.if_stack_torch(g, dev) for g in cfg.grids]
    wfs = [synim.Wfs.from_numpy(P, cfg.p, v, device=dev) for P, v in zip(cfg.pupils, cfg.valids)]
    n_out = cfg.n_sub * cfg.p
    maps = [synim.affine_from_geometry(pr.geometry, 512, 512, n_out, n_out) for pr in cfg.pairs]
    B = synim.Batch(wfs, stacks, [(pr.wfs, pr.dm, A) for pr, A in zip(cfg.pairs, maps)], device=dev)
    tuned = B.autotune(6)
    cfg_b = B.config()
    cfg_b["parts"] = B.parts()
    ms = _event_ms(B.run_graph, reps)
    if B.status() != 0:
        raise RuntimeError("MCAO batch plan status non-zero")
    byts = 0
    cols = 0
    for d, g in enumerate(cfg.grids):
        U = np.zeros((512, 512), bool)
        for pr, A in zip(cfg.pairs, maps):
            if pr.dm == d:
                U |= touched_mask(cfg.pupils[pr.wfs], cfg.p, cfg.valids[pr.wfs], A, 512)
                byts += 8 * len(cfg.valids[pr.wfs]) * g.n_act
                cols += g.n_act
        byts += 4 * int(U.sum()) * g.n_act
    B.close()
    del stacks
    torch.cuda.empty_cache()
    return {"workload": "MCAO 6 LGS WFS x 3 DMs (81^2/47^2/37^2 on 512^2), 68x68 subap x 7 px, "
                        "18 pair maps, one persistent launch per patch size (hipGraph replay)",
            "ms_per_batch": ms, "im_columns": cols, "columns_per_s": cols / (ms * 1e-3),
            "algorithmic_bytes": byts, "achieved_GBs": byts / (ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": byts / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "traffic": stored_traffic(MCAO_TRAFFIC_FILE),
            "config": cfg_b, "autotune_ms": tuned}


def elt_engine_legs(synim, dev, cfg, Fd, A, wfs, launch_bytes, reps: int = 10):
    """Two more builds of the ELT SCAO workload on its resident IF stack, plan
    + stream per call: the telescoping-sum slope engine, and the edge-repaired
    build of the same stack pre-masked (in place, so it runs last) by a DM-side
    annulus 4 px inside the pupil's outer edge and 4 px outside its central
    obscuration (the repair restores the samples the mask edge corrupts)."""
    import torch
    import workloads as wl
    n_act = cfg.grid.n_act
    ws = torch.empty(synim.im_workspace_bytes(wfs, A, 1), dtype=torch.uint8, device=dev)
    out = torch.empty((n_act, 2 * cfg.n_valid), dtype=torch.float32, device=dev)
    ms_t = _event_ms(lambda: synim.im_build_tsum(Fd, A, wfs, out=out, ws=ws), reps)
    M = wl.pupil_mask(512, 472.0, (0.28 * 480.0 + 8.0) / 472.0)
    Md = torch.from_numpy(M).to(dev)
    Fd.mul_(Md.to(torch.float32))
    del ws
    ms_r = _event_ms(lambda: synim.im_build_repaired(Fd, Md, A, wfs, out=out), reps)
    return {"tsum": {"workload": "ELT SCAO IM, telescoping-sum slope engine (plan + stream)",
                     "ms_per_build": ms_t, "columns_per_s": n_act / (ms_t * 1e-3),
                     "frac_of_hbm_peak": launch_bytes / (ms_t * 1e-3) / 1e9 / PEAK_HBM_GBS},
            "repair": {"workload": "ELT SCAO IM of the IF stack pre-masked by a DM-side annulus, "
                                   "with edge repair (plan + stream)",
                       "ms_per_build": ms_r, "columns_per_s": n_act / (ms_r * 1e-3),
                       "frac_of_hbm_peak": launch_bytes / (ms_r * 1e-3) / 1e9 / PEAK_HBM_GBS}}


def standalone_legs(synim, dev, cfg, Fd, A, wfs, reps: int = 5):
    """The two standalone steps on the ELT stack: the warp of every IF onto the
    haloed 482^2 WFS window (reads the source pixels the window's bilinear
    taps touch, writes the window), then the slopes of the warped stack
    (reads every haloed sample, writes the IM).  Algorithmic bytes from the
    geometry; HIP events."""
    import numpy as np
    import torch
    n_act, H = cfg.grid.n_act, cfg.n_out
    Hh = H + 2
    warped = torch.empty((n_act, Hh, Hh), dtype=torch.float32, device=dev)
    ms_w = _event_ms(lambda: synim.affine_warp(Fd, A, H, H, halo=1, out=warped), reps)
    ys, xs = np.mgrid[-1:H + 1, -1:H + 1].astype(np.float64)
    sx = A[0, 0] * xs + A[0, 1] * ys + A[0, 2]
    sy = A[1, 0] * xs + A[1, 1] * ys + A[1, 2]
    i, j = np.floor(sx).astype(np.int64), np.floor(sy).astype(np.int64)
    T = np.zeros((512, 512), bool)
    for di in (0, 1):
        for dj in (0, 1):
            ok = (i + di >= 0) & (i + di < 512) & (j + dj >= 0) & (j + dj < 512)
            T[(j + dj)[ok], (i + di)[ok]] = True
    wb = (4 * int(T.sum()) + 4 * Hh * Hh) * n_act
    out = torch.empty((n_act, 2 * cfg.n_valid), dtype=torch.float32, device=dev)
    ms_s = _event_ms(lambda: synim.sa_slopes(warped, wfs, out=out), reps)
    sb = (4 * Hh * Hh + 8 * cfg.n_valid) * n_act
    del warped
    torch.cuda.empty_cache()
    return {"warp": {"workload": "synim_affine_warp: 5257 ELT IFs onto the haloed 482^2 window",
                     "ms": ms_w, "algorithmic_bytes": wb,
                     "frac_of_hbm_peak": wb / (ms_w * 1e-3) / 1e9 / PEAK_HBM_GBS},
            "slopes": {"workload": "synim_sa_slopes: 5257 warped 482^2 maps -> the ELT IM",
                       "ms": ms_s, "algorithmic_bytes": sb,
                       "frac_of_hbm_peak": sb / (ms_s * 1e-3) / 1e9 / PEAK_HBM_GBS}}


def modal_leg(synim, dev, reps: int = 10):
    """Modal IM under the full composite: 4519 Fourier modes (up to 38 cycles
    per 480-px meta-pupil) on 512^2, one LGS WFS of the MCAO system (68x68
    subapertures of 7 px, clocked 15 deg, anamorphic magnification 1.00 x 0.97)
    at the 4-km DM's cone and footprint, the DM misregistered.  Plan + stream
    per build; algorithmic bytes as the SCAO build's (touched IF pixels x
    modes + the IM)."""
    import torch
    import workloads as wl
    cfg = wl.mcao(0)
    n_out = cfg.n_sub * cfg.p
    g = cfg.pairs[4].geometry
    g.wfs_mag_x, g.wfs_mag_y = 1.0, 0.97
    g.dm_shift_x, g.dm_shift_y, g.dm_rot, g.dm_mag = 0.37, -0.23, math.radians(0.3), 1.003
    modes = wl.fourier_modes(4519)
    F = wl.fourier_stack_torch(modes, 512, 480.0, dev)
    A = synim.affine_from_geometry(g, 512, 512, n_out, n_out)
    P, v = cfg.pupils[1], cfg.valids[1]
    wfs = synim.Wfs.from_numpy(P, cfg.p, v, device=dev)
    ws = torch.empty(synim.im_workspace_bytes(wfs, A, 1), dtype=torch.uint8, device=dev)
    out = torch.empty((len(modes), 2 * len(v)), dtype=torch.float32, device=dev)
    synim.im_autotune(F, A, wfs, max_candidates=16, ws=ws)

    def step():
        synim.im_plan(wfs, A, ws=ws, grid=(512, 512))
        synim.im_apply(F, A, wfs, ws, out=out)
    ms = _event_ms(step, reps)
    S = int(touched_mask(P, cfg.p, v, A, 512).sum())
    byts = (4 * S + 8 * len(v)) * len(modes)
    del F
    torch.cuda.empty_cache()
    return {"workload": "modal IM: 4519 Fourier modes on 512^2, LGS WFS 68x68 x 7 px, composite "
                        "map with cone, footprint, DM misregistration, WFS clocking and "
                        "anamorphosis",
            "ms_per_build": ms, "im_columns": len(modes),
            "columns_per_s": len(modes) / (ms * 1e-3), "algorithmic_bytes": byts,
            "achieved_GBs": byts / (ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": byts / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "config": synim.im_config(wfs, A)}


PEAK_F64_MFMA_TFS = 78.6


def projection_leg(synim, dev):
    """Tomographic projection P_opt (Sec. 2.5) at the MCAO scale: the 3 DMs
    (8171 IFs on 512^2 at 8.19 cm/px) and 3 virtual layers (2, 8, 16 km; 4083
    Gaussian modes) over 9 directions (3x3 grid, 40 arcsec pitch), the 476-px
    pupil binned 4x4 (94 104 rows).  The dominant kernel is the FP64 MFMA GEMM
    of the Gram matrix (timed alone on the full square: 2 rows n^2 flops)."""
    import numpy as np
    import torch
    import workloads as wl
    cfg = wl.mcao(0)
    pix = cfg.pixel_scale_m
    dms = [(wl.if_stack_torch(g, dev), h, pix) for g, h in zip(cfg.grids, cfg.altitudes_m)]
    lgrids = [wl.actuator_grid(41, 12.0, 512, keep_radius=250.0) for _ in range(3)]
    layers = [(wl.if_stack_torch(g, dev), h, pix) for g, h in zip(lgrids, (2000.0, 8000.0,
                                                                          16000.0))]
    a = math.radians(40.0 / 3600.0)
    dirs = np.array([[x * a, y * a] for y in (-1, 0, 1) for x in (-1, 0, 1)])
    pupil = wl.pupil_mask(476, 476.0, 0.28)
    Pt = synim.proj_matrix(dms, dirs, pupil, pix, bin=4)
    n, rows = Pt.shape
    G = torch.empty((n, n), dtype=torch.float64, device=dev)
    gemm_ms = _event_ms(lambda: synim.gemm_f64(n, n, rows, 1.0, Pt, 1, rows, Pt, 1, rows, 0.0,
                                               G, n), 2)
    lam = float((Pt * Pt).sum(dim=1).mean()) * 1e-3
    del G, Pt
    torch.cuda.empty_cache()
    ws = torch.empty(synim.proj_workspace_bytes(dms, layers, len(dirs), pupil, 4),
                     dtype=torch.uint8, device=dev)
    opt_ms = _event_ms(lambda: synim.proj_opt(dms, layers, dirs, pupil, pix, lam, bin=4, ws=ws), 2)
    flops = 2.0 * rows * n * n
    del ws, dms, layers
    torch.cuda.empty_cache()
    return {"workload": "P_opt: 3 DMs (8171 IFs) x 3 layers (4083 modes), 9 directions, 476-px "
                        "pupil binned 4x4 (94104 rows), FP64",
            "p_opt_ms": opt_ms, "gram_gemm_ms": gemm_ms, "gram_gemm_flops": flops,
            "roofline": {"bound": "mfma", "achieved": flops / (gemm_ms * 1e-3) / 1e12,
                         "peak": PEAK_F64_MFMA_TFS, "unit": "TFLOP/s",
                         "frac": flops / (gemm_ms * 1e-3) / 1e12 / PEAK_F64_MFMA_TFS}}


def jacobian_leg(synim, dev, reps: int = 50):
    """Adjoint workload: 8x8 SCAO, 81 IFs; IM + 4 Jacobian planes, and the VJP."""
    import numpy as np
    import torch
    import workloads as wl
    cfg = wl.scao_small()
    F = torch.from_numpy(wl.if_stack(cfg.grid)).to(dev)
    A, dA = synim.affine_from_misreg(cfg.theta, 96, 96, 80, 80)
    wfs = synim.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid, device=dev)
    ws = torch.empty(synim.im_workspace_bytes(wfs, A, 5), dtype=torch.uint8, device=dev)
    g = torch.from_numpy(np.random.default_rng(0).standard_normal((81, 2 * cfg.n_valid))
                         .astype(np.float32)).to(dev)
    jac = _event_ms(lambda: synim.im_jacobian(F, A, dA, wfs, with_im=True, ws=ws), reps)
    vjp = _event_ms(lambda: synim.im_vjp(F, A, dA, wfs, g, ws=ws), reps)
    im = _event_ms(lambda: synim.im_build(F, A, wfs, ws=ws), reps)
    return {"workload": "8x8 SCAO (81 IFs on 96^2): plan + stream, per call",
            "im_us": im * 1e3, "im_plus_jacobian_us": jac * 1e3, "vjp_us": vjp * 1e3}


def misreg_leg(n_train: int, n_eval: int, epochs: int):
    """Learned misregistration estimate vs Gauss-Newton (training set, network
    training and evaluation all on the GPU kernels)."""
    from paper_2606_07759_amd import learned
    rep = learned.run(n_train=n_train, n_eval=n_eval, epochs=epochs,
                      log=lambda m: log("misreg:", m))
    rep["workload"] = ("20 Zernike probes (Noll 2-21) on the 8x8 SCAO WFS, MLP 2x4000->512->256->4, "
                       f"{n_train} training samples, {n_eval} held-out seeds")
    return rep


def schedules_leg(index: int = -1, reps: int = 10):
    """The ELT stream kernel under its two schedules: every one-chunk-per-XCD
    candidate and the dynamic candidates of the same tile shapes, each pinned,
    planned and timed over `reps` launches (HIP events on the launch stream).
    index >= 0 runs only that entry of the list (for a counter pass)."""
    import torch
    import paper_2606_07759_amd as synim
    import workloads as wl
    synim.load()
    dev = torch.device("cuda:0")
    cfg = wl.scao_elt(0)
    Fd = wl.if_stack_torch(cfg.grid, dev)
    A, _ = synim.affine_from_misreg(cfg.theta, 512, 512, cfg.n_out, cfg.n_out)
    wfs = synim.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid, device=dev)
    launch_bytes = cfg.grid.n_act * (4 * touched_if_pixels(cfg, A) + 8 * cfg.n_valid)
    shape = lambda c: tuple(c[k] for k in synim._CFG_KEYS if k != "schedule")
    cands = synim.im_candidates(wfs, A)
    xcd_shapes = {shape(c) for c in cands if c["schedule"] != 0}
    sel = [c for c in cands if shape(c) in xcd_shapes]
    ws = torch.empty(synim.im_workspace_bytes(wfs, A, 1), dtype=torch.uint8, device=dev)
    out = torch.empty((cfg.grid.n_act, 2 * cfg.n_valid), dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream()
    for i, c in enumerate(sel):
        if index >= 0 and i != index:
            continue
        synim.im_set_config(wfs, A, c)
        synim.im_plan(wfs, A, ws=ws, grid=(cfg.grid.grid_n, cfg.grid.grid_n))
        for _ in range(3):
            synim.im_apply(Fd, A, wfs, ws, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            synim.im_apply(Fd, A, wfs, ws, out=out)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"index": i, "ms": round(ms, 4),
                          "frac": round(launch_bytes / (ms * 1e-3) / 8e12, 4),
                          "status": synim.plan_status(ws), **c}), flush=True)
    synim.autotune_clear()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tune", type=int, default=32,
                    help="stream-kernel configurations the autotuner times before the run")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the MCAO, Jacobian and misregistration legs")
    ap.add_argument("--misreg-train", type=int, default=50_000)
    ap.add_argument("--misreg-eval", type=int, default=1000)
    ap.add_argument("--misreg-epochs", type=int, default=60)
    ap.add_argument("--misreg-replay", action="store_true",
                    help="only replay the three misregistration estimate modes at batch 1 "
                         "(the workload of the fit's kernel trace)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--misreg-only", action="store_true",
                    help="only run the learned-misregistration leg (sizes from --misreg-train, "
                         "--misreg-eval, --misreg-epochs) and print its figures")
    ap.add_argument("--mcao-only", action="store_true",
                    help="only run the MCAO batch leg (the workload of its kernel trace) and "
                         "print its figures")
    ap.add_argument("--schedules", type=int, nargs="?", const=-1, default=None,
                    metavar="INDEX",
                    help="only time the ELT stream kernel under the dynamic and the "
                         "one-chunk-per-XCD schedules (INDEX: one entry only)")
    ap.add_argument("--standalone-only", action="store_true",
                    help="only run the standalone warp and slopes legs on the ELT stack (the "
                         "workload of their kernel trace) and print their figures")
    args = ap.parse_args()
    if args.standalone_only:
        import torch
        import paper_2606_07759_amd as synim
        import workloads as wl
        synim.load()
        dev = torch.device("cuda:0")
        cfg = wl.scao_elt(args.seed)
        Fd = wl.if_stack_torch(cfg.grid, dev)
        A, _ = synim.affine_from_misreg(cfg.theta, 512, 512, cfg.n_out, cfg.n_out)
        wfs = synim.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid, device=dev)
        print(json.dumps(standalone_legs(synim, dev, cfg, Fd, A, wfs)), flush=True)
        return
    if args.schedules is not None:
        schedules_leg(args.schedules)
        return
    if args.copy_probe:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": src.numel() * 4,
                          "copy_probe_bytes_written": dst.numel() * 4}), flush=True)
        return
    if args.misreg_replay:
        from paper_2606_07759_amd import learned
        learned.replay_fits()
        return
    if args.misreg_only:
        print(json.dumps(misreg_leg(args.misreg_train, args.misreg_eval, args.misreg_epochs)),
              flush=True)
        return
    if args.mcao_only:
        import paper_2606_07759_amd as synim
        synim.load()
        import torch
        print(json.dumps(mcao_leg(synim, torch.device("cuda:0"))), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the IM build shards by actuator columns with no "
              "exchange, so only --gpus 1 is run here", file=sys.stderr)
        sys.exit(2)

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.seed, args.cpu_seconds)

    import numpy as np
    import torch
    import paper_2606_07759_amd as synim
    import workloads as wl

    synim.load()
    dev = torch.device("cuda:0")
    cfg = wl.scao_elt(args.seed)
    n_act, H = cfg.grid.n_act, cfg.n_out
    log(f"generating {n_act} IFs of {cfg.grid.grid_n}^2 on the device")
    Fd = wl.if_stack_torch(cfg.grid, dev)
    A, _ = synim.affine_from_misreg(cfg.theta, 512, 512, H, H)
    wfs = synim.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid, device=dev)
    ws = torch.empty(synim.im_workspace_bytes(wfs, A, 1), dtype=torch.uint8, device=dev)
    out = torch.empty((n_act, 2 * cfg.n_valid), dtype=torch.float32, device=dev)

    S = touched_if_pixels(cfg, A)
    bytes_per_col = 4 * S + 8 * cfg.n_valid
    launch_bytes = bytes_per_col * n_act

    log("autotuning the stream kernel")
    tune_ms = synim.im_autotune(Fd, A, wfs, max_candidates=args.tune, ws=ws)
    chosen = synim.im_config(wfs, A)
    log(f"chosen {chosen} ({min(tune_ms):.3f} ms best of {len(tune_ms)})")
    for _ in range(args.warmup):
        synim.im_plan(wfs, A, ws=ws, grid=(512, 512))
        synim.im_apply(Fd, A, wfs, ws, out=out)
    torch.cuda.synchronize()
    if synim.plan_status(ws) != 0:
        raise RuntimeError("plan status non-zero")
    log(f"warmup done; timing {args.steps} steps")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        synim.im_plan(wfs, A, ws=ws, grid=(512, 512))
        synim.im_apply(Fd, A, wfs, ws, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    # The stream kernel's own duration: HIP events on its launch stream around
    # each apply, in a second pass of the same steps.  Each timed event record
    # puts about 5.6 us between the kernels around it, so the throughput pass
    # above records none.
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    for k in range(args.steps):
        synim.im_plan(wfs, A, ws=ws, grid=(512, 512))
        ev[k][0].record()
        synim.im_apply(Fd, A, wfs, ws, out=out)
        ev[k][1].record()
    torch.cuda.synchronize()
    apply_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    achieved = launch_bytes / (apply_ms * 1e-3) / 1e9
    traffic = stored_traffic(TRAFFIC_FILE)
    legs = {}
    if not args.no_legs:
        log("legs: standalone warp and slopes")
        legs.update(standalone_legs(synim, dev, cfg, Fd, A, wfs))
        log("legs: telescoping-sum engine, edge repair")
        legs.update(elt_engine_legs(synim, dev, cfg, Fd, A, wfs, launch_bytes))
    del Fd
    torch.cuda.empty_cache()
    if not args.no_legs:
        log("leg: MCAO batch")
        legs["mcao_batch"] = mcao_leg(synim, dev)
        log("leg: modal IM")
        legs["modal_im"] = modal_leg(synim, dev)
        log("leg: tomographic projection")
        legs["projection"] = projection_leg(synim, dev)
        log("leg: Jacobian / VJP")
        legs["adjoint"] = jacobian_leg(synim, dev)
        log("leg: learned misregistration vs Gauss-Newton")
        legs["misreg_fit"] = misreg_leg(args.misreg_train, args.misreg_eval, args.misreg_epochs)
    rec = {
        "metric": METRIC,
        "value": n_act / (ms_step * 1e-3),
        "unit": "IM columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ELT SCAO IM: 80x80 subap x 6 px, 480-px pupil 28% obscured, "
                               f"{n_act} Gaussian IFs on 512^2, seed {args.seed}",
                   "n_act": n_act, "n_valid": cfg.n_valid, "if_grid": 512,
                   "theta": [float(v) for v in cfg.theta], "kernel_config": chosen},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic},
        "cpu_baseline": cpu,
        "detail": {"stream_kernel_ms": apply_ms, "plan_plus_stream_ms": ms_step,
                   "algorithmic_bytes_per_column": bytes_per_col,
                   "touched_if_pixels_per_column": S, "algorithmic_bytes_per_launch": launch_bytes},
        "legs": legs,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
