"""FP64 oracle IM columns of the full-size workloads, computed in a pool of host
processes (test infrastructure: the oracle itself is unchanged, it only runs
over many columns at once).

Each worker regenerates the influence functions it needs from the seeded
workload description (input synthesis, shared with the GPU side) and calls
``oracle.im.im_build`` on them.
"""
from __future__ import annotations

import concurrent.futures as cf
import multiprocessing as mp
import os

import numpy as np

CHUNK = 12


def workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _elt_job(args):
    seed, cols, A = args
    import workloads as wl
    from oracle import im as oim
    cfg = wl.scao_elt(seed)
    F = np.stack([wl.if_single(cfg.grid, a) for a in cols])
    return oim.im_build(F, A[:, :2], A[:, 2], cfg.pupil, cfg.p, cfg.valid)


def _mcao_job(args):
    seed, pair, cols, A = args
    import workloads as wl
    from oracle import im as oim
    cfg = wl.mcao(seed)
    pr = cfg.pairs[pair]
    g = cfg.grids[pr.dm]
    F = np.stack([wl.if_single(g, a) for a in cols])
    return oim.im_build(F, A[:, :2], A[:, 2], cfg.pupils[pr.wfs], cfg.p, cfg.valids[pr.wfs])


def _run(fn, jobs):
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=workers(), mp_context=ctx) as ex:
        return list(ex.map(fn, jobs))


def elt_columns(seed: int, cols, A) -> np.ndarray:
    """Oracle IM rows [len(cols)][2N] of the ELT SCAO workload (seed) under map A."""
    cols = list(cols)
    jobs = [(seed, cols[i:i + CHUNK], np.asarray(A)) for i in range(0, len(cols), CHUNK)]
    return np.concatenate(_run(_elt_job, jobs))


def mcao_columns(seed: int, pair_cols, maps) -> list:
    """Oracle IM rows of the MCAO workload: pair_cols = [(pair, [cols])], maps per pair."""
    jobs, owner = [], []
    for pair, cols in pair_cols:
        cols = list(cols)
        for i in range(0, len(cols), CHUNK):
            jobs.append((seed, pair, cols[i:i + CHUNK], np.asarray(maps[pair])))
            owner.append(pair)
    res = _run(_mcao_job, jobs)
    out = {}
    for pair, r in zip(owner, res):
        out.setdefault(pair, []).append(r)
    return [np.concatenate(out[pair]) for pair, _ in pair_cols]


def oracle_gn_sample(seed: int, max_iter: int = 20, tol: float = 1e-6):
    """FP64 oracle Gauss-Newton on one learned-fit sample, its measured slopes
    synthesised by the oracle from the seed (labels, SNR and noise as the
    workload draws them).  Returns (theta, iterations, converged, truth)."""
    import workloads as wl
    from oracle import misreg as omr
    pc = wl.probe_config()
    cfg = pc.scao
    maps = pc.probe_maps.astype(np.float64)
    scale = 0.5 * (wl.LABEL_HI - wl.LABEL_LO)
    th, snr, rng = wl.draw_misreg_labels(int(seed))
    S = omr.probe_slopes(maps, th, cfg.pupil, cfg.p, cfg.valid).ravel()
    noise = rng.standard_normal(S.size).astype(np.float32).astype(np.float64)
    meas = S + noise * np.sqrt(np.mean(S * S)) / snr
    t, it, ok = omr.gauss_newton(meas, maps, cfg.pupil, cfg.p, cfg.valid, scale,
                                 max_iter=max_iter, tol=tol)
    return t, it, ok, th
