"""Every column of the full-size builds against the FP64 oracle.

* ELT SCAO (5257 IFs of 512^2, 80x80 subapertures of 6 px): the stream kernel
  configuration is autotuned exactly as the benchmark does it, then ALL 5257
  IM columns are compared with the oracle (computed column by column in a pool
  of host processes).  A failure that hits a different random set of actuators
  on each run cannot hide behind a sample.
* MCAO batch (6 LGS WFS x 3 DMs, 18 pairs): after the batch autotuner, one
  column of every actuator chunk of every pair (a random actuator inside each
  chunk of 64, plus the first and last actuator), i.e. every XCD queue and
  every chunk boundary of the persistent launch.

Tolerance: max|dIM| <= 1e-5 * max|IM| over the compared columns.
"""
import sys

import numpy as np
import pytest

import oracle_pool
import workloads as wl

pytestmark = pytest.mark.gpu
IM_TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def test_elt_every_column_autotuned(gpu_lib):
    import torch
    S = gpu_lib
    cfg = wl.scao_elt(0)
    say("[case] elt all columns: generating", cfg.grid.n_act, "IFs")
    Fd = wl.if_stack_torch(cfg.grid, "cuda")
    A, _ = S.affine_from_misreg(cfg.theta, 512, 512, 480, 480)
    wfs = S.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid)
    ws = torch.empty(S.im_workspace_bytes(wfs, A, 1), dtype=torch.uint8, device="cuda")
    S.im_autotune(Fd, A, wfs, max_candidates=32, ws=ws)
    say("[case] elt all columns: config", S.im_config(wfs, A))
    S.im_plan(wfs, A, ws=ws, grid=(512, 512))
    assert S.plan_status(ws) == 0
    assert S.plan_oob(ws) == 0
    im = S.im_apply(Fd, A, wfs, ws).cpu().numpy()
    del Fd
    torch.cuda.empty_cache()
    say("[case] elt all columns: oracle on", oracle_pool.workers(), "processes")
    ref = oracle_pool.elt_columns(0, range(cfg.grid.n_act), A)
    e = rel_err(im, ref)
    worst = np.max(np.abs(im - ref), axis=1)
    say("[case] elt all columns: rel err", e, "worst column", int(np.argmax(worst)))
    assert e <= IM_TOL, (e, np.flatnonzero(worst > IM_TOL * np.abs(ref).max())[:20])


def test_mcao_every_chunk_of_every_pair(gpu_lib):
    import torch
    S = gpu_lib
    cfg = wl.mcao(0)
    say("[case] mcao chunks: generating", [g.n_act for g in cfg.grids])
    stacks = [wl.if_stack_torch(g, "cuda") for g in cfg.grids]
    wfs = [S.Wfs.from_numpy(P, cfg.p, v) for P, v in zip(cfg.pupils, cfg.valids)]
    n_out = cfg.n_sub * cfg.p
    maps = [S.affine_from_geometry(pr.geometry, 512, 512, n_out, n_out) for pr in cfg.pairs]
    B = S.Batch(wfs, stacks, [(pr.wfs, pr.dm, A) for pr, A in zip(cfg.pairs, maps)])
    B.autotune(6)
    B.run_graph()
    torch.cuda.synchronize()
    assert B.status() == 0
    assert B.oob() == 0
    say("[case] mcao chunks: config", B.config())
    rng = np.random.default_rng(11)
    pair_cols = []
    for i, pr in enumerate(cfg.pairs):
        n = cfg.grids[pr.dm].n_act
        cols = {0, n - 1}
        for c0 in range(0, n, 64):
            cols.add(int(rng.integers(c0, min(n, c0 + 64))))
        pair_cols.append((i, sorted(cols)))
    got = [B.outs[i][cols].cpu().numpy() for i, cols in pair_cols]
    B.close()
    del stacks
    torch.cuda.empty_cache()
    say("[case] mcao chunks: oracle on", sum(len(c) for _, c in pair_cols), "columns")
    refs = oracle_pool.mcao_columns(0, pair_cols, maps)
    worst = 0.0
    for (i, cols), g, r in zip(pair_cols, got, refs):
        e = rel_err(g, r)
        worst = max(worst, e)
        assert e <= IM_TOL, (i, e)
    say("[case] mcao chunks: worst rel err", worst)
