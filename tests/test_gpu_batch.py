"""GPU parity of the multi-pair batched build (the paper's multi-WFS batch).

* a small multi-WFS x multi-DM system (uneven valid-subaperture and actuator
  counts, per-pair cone scale / footprint / clocking): every pair's IM against
  the FP64 oracle and against the single-pair build;
* hipGraph replays, with eager work and synchronisations between them, each
  checked against the eager result; new maps uploaded to device memory and
  replayed without re-capture;
* the batch autotuner keeps results within tolerance;
* a batch split by patch size (one part per patch, each its own launch):
  parity, graph replays, new maps, autotuning and refused maps;
* the full 6 LGS x 3 DM MCAO workload on sampled columns of every pair.
"""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import geometry as og, im as oim

pytestmark = pytest.mark.gpu
IM_TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def S(gpu_lib):
    return gpu_lib


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def small_system(seed=3):
    """3 WFS (12x12 subapertures of 5 px, shifted pupils) x 2 DMs."""
    rng = wl.rng_for(seed)
    wfs = []
    for w in range(3):
        off = (float(rng.uniform(-2, 2)), float(rng.uniform(-2, 2)))
        P = wl.pupil_mask(60, 60.0, 0.25, off)
        wfs.append((P, wl.valid_subapertures(P, 5)))
    grids = [wl.actuator_grid(9, 7.5, 80, keep_radius=37.0), wl.actuator_grid(6, 12.0, 80)]
    pairs = []
    for w in range(3):
        for d, h in enumerate((0.0, 8e3)):
            az = math.radians(120 * w)
            g = wl.Geometry(cone_scale=1 - h / 90e3, footprint_x=h * 2e-4 * math.cos(az),
                            footprint_y=h * 2e-4 * math.sin(az), wfs_rot=math.radians(10 * w - 10))
            pairs.append((w, d, g))
    return wfs, grids, pairs


def test_small_batch_parity_and_graph(S):
    import torch
    wfs_np, grids, pairs = small_system()
    wfs = [S.Wfs.from_numpy(P, 5, v) for P, v in wfs_np]
    stacks_np = [wl.if_stack(g) for g in grids]
    stacks = [torch.from_numpy(F).cuda() for F in stacks_np]
    maps = [S.affine_from_geometry(g, 80, 80, 60, 60) for (_, _, g) in pairs]
    B = S.Batch(wfs, stacks, [(w, d, A) for (w, d, _), A in zip(pairs, maps)])
    assert B.status() == 0
    outs = [o.clone() for o in B.run()]
    torch.cuda.synchronize()
    assert B.status() == 0
    for i, (w, d, g) in enumerate(pairs):
        P, v = wfs_np[w]
        A = maps[i]
        ref = oim.im_build(stacks_np[d], A[:, :2], A[:, 2], P, 5, v)
        got = outs[i].cpu().numpy()
        assert rel_err(got, ref) <= IM_TOL, (i, rel_err(got, ref))
        single = S.im_build(stacks[d], A, wfs[w]).cpu().numpy()
        assert np.max(np.abs(single - got)) <= IM_TOL * np.abs(ref).max()
    # graph replays interleaved with eager work: every replay equals eager
    for rep in range(3):
        for o in B.outs:
            o.fill_(-7.0)
        B.run_graph()
        torch.cuda.synchronize()
        for i in range(len(pairs)):
            assert torch.equal(B.outs[i], outs[i]), (rep, i)
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        del junk
    # new maps in device memory, replayed without re-capture
    maps2 = [S.affine_from_geometry(
        wl.Geometry(cone_scale=g.cone_scale, footprint_x=g.footprint_x + 0.7,
                    footprint_y=g.footprint_y - 0.4, wfs_rot=g.wfs_rot + 0.003), 80, 80, 60, 60)
        for (_, _, g) in pairs]
    B.set_maps(maps2)
    B.run_graph()
    torch.cuda.synchronize()
    assert B.status() == 0
    for i, (w, d, g) in enumerate(pairs):
        P, v = wfs_np[w]
        A = maps2[i]
        ref = oim.im_build(stacks_np[d], A[:, :2], A[:, 2], P, 5, v)
        assert rel_err(B.outs[i].cpu().numpy(), ref) <= IM_TOL, i
    B.close()


def split_system():
    """2 WFS x 2 DMs whose pairs need different patches: WFS 0 unclocked behind
    a 0.9 cone scale (8x8 patches), WFS 1 clocked by 45 deg (12x12)."""
    wfs_np, grids, _ = small_system(seed=7)
    pairs = []
    for w, (rot, cone) in enumerate(((0.0, 0.9), (45.0, 1.0))):
        for d in range(2):
            pairs.append((w, d, wl.Geometry(cone_scale=cone, footprint_x=0.3 * d,
                                             wfs_rot=math.radians(rot))))
    return wfs_np[:2], grids, pairs


def test_split_batch_by_patch_size(S):
    """A batch whose pairs' patches differ enough runs as one part per patch
    size: parity with the oracle, graph replays, new maps, the autotuner, and
    a map that outgrows its part's patch refused."""
    import torch
    wfs_np, grids, pairs = split_system()
    wfs = [S.Wfs.from_numpy(P, 5, v) for P, v in wfs_np]
    stacks_np = [wl.if_stack(g) for g in grids]
    stacks = [torch.from_numpy(F).cuda() for F in stacks_np]
    maps = [S.affine_from_geometry(g, 80, 80, 60, 60) for (_, _, g) in pairs]
    B = S.Batch(wfs, stacks, [(w, d, A) for (w, d, _), A in zip(pairs, maps)])
    assert B.parts() == 2
    outs = [o.clone() for o in B.run()]
    torch.cuda.synchronize()
    assert B.status() == 0
    for i, (w, d, g) in enumerate(pairs):
        P, v = wfs_np[w]
        A = maps[i]
        ref = oim.im_build(stacks_np[d], A[:, :2], A[:, 2], P, 5, v)
        assert rel_err(outs[i].cpu().numpy(), ref) <= IM_TOL, (i, rel_err(outs[i].cpu().numpy(), ref))
    for rep in range(3):
        for o in B.outs:
            o.fill_(-7.0)
        B.run_graph()
        torch.cuda.synchronize()
        for i in range(len(pairs)):
            assert torch.equal(B.outs[i], outs[i]), (rep, i)
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        del junk
    maps2 = [S.affine_from_geometry(
        wl.Geometry(cone_scale=g.cone_scale, footprint_x=g.footprint_x + 0.6,
                    footprint_y=-0.5, wfs_rot=g.wfs_rot + 0.002), 80, 80, 60, 60)
        for (_, _, g) in pairs]
    B.set_maps(maps2)
    B.run_graph()
    torch.cuda.synchronize()
    assert B.status() == 0
    for i, (w, d, g) in enumerate(pairs):
        P, v = wfs_np[w]
        A = maps2[i]
        ref = oim.im_build(stacks_np[d], A[:, :2], A[:, 2], P, 5, v)
        assert rel_err(B.outs[i].cpu().numpy(), ref) <= IM_TOL, i
    ref2 = [o.clone() for o in B.outs]
    times = B.autotune(3)
    assert len(times) >= 1 and all(t > 0 for t in times)
    got = B.run()
    torch.cuda.synchronize()
    for a, b in zip(got, ref2):
        assert torch.max(torch.abs(a - b)).item() <= IM_TOL * torch.max(torch.abs(b)).item()
    # WFS 0's pairs clocked by 45 deg outgrow the 8x8 patches of their part
    maps3 = [S.affine_from_geometry(
        wl.Geometry(cone_scale=g.cone_scale, footprint_x=g.footprint_x, wfs_rot=math.radians(45.0)),
        80, 80, 60, 60) for (_, _, g) in pairs]
    with pytest.raises(S.SynimError) as ei:
        B.set_maps(maps3)
    assert ei.value.status == -8
    B.close()


def test_batch_autotune_keeps_results(S):
    import torch
    wfs_np, grids, pairs = small_system(seed=5)
    wfs = [S.Wfs.from_numpy(P, 5, v) for P, v in wfs_np]
    stacks = [torch.from_numpy(wl.if_stack(g)).cuda() for g in grids]
    maps = [S.affine_from_geometry(g, 80, 80, 60, 60) for (_, _, g) in pairs]
    B = S.Batch(wfs, stacks, [(w, d, A) for (w, d, _), A in zip(pairs, maps)])
    ref = [o.clone() for o in B.run()]
    times = B.autotune(4)
    assert len(times) >= 1 and all(t > 0 for t in times)
    got = B.run()
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.max(torch.abs(a - b)).item() <= IM_TOL * torch.max(torch.abs(b)).item()
    B.close()


def test_mcao_full_size_sampled(S):
    import torch
    cfg = wl.mcao(0)
    say("mcao: generating", [g.n_act for g in cfg.grids])
    stacks = [wl.if_stack_torch(g, "cuda") for g in cfg.grids]
    wfs = [S.Wfs.from_numpy(P, cfg.p, v) for P, v in zip(cfg.pupils, cfg.valids)]
    maps = [S.affine_from_geometry(pr.geometry, 512, 512, 476, 476) for pr in cfg.pairs]
    B = S.Batch(wfs, stacks, [(pr.wfs, pr.dm, A) for pr, A in zip(cfg.pairs, maps)])
    B.run()
    torch.cuda.synchronize()
    assert B.status() == 0
    say("mcao: built", B.config())
    rng = np.random.default_rng(1)
    worst = 0.0
    for i, pr in enumerate(cfg.pairs):
        g = cfg.grids[pr.dm]
        cols = sorted(rng.choice(g.n_act, 2, replace=False).tolist())
        Fs = np.stack([wl.if_single(g, a) for a in cols])
        A = maps[i]
        ref = oim.im_build(Fs, A[:, :2], A[:, 2], cfg.pupils[pr.wfs], cfg.p, cfg.valids[pr.wfs])
        got = B.outs[i][cols].cpu().numpy()
        worst = max(worst, rel_err(got, ref))
    say("mcao: worst rel err", worst)
    assert worst <= IM_TOL
    B.close()
    del stacks
