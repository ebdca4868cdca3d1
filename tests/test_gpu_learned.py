"""GPU parity of the learned-misregistration path against the FP64 oracle.

* MLP kernels (forward, MSE backward, Adam) against the oracle's FP64 net on
  the same parameters and inputs, through both forward code paths (small
  batches, and matrix-core GEMMs with ragged tiles and split-K products):
  outputs and gradients within 1e-4 of their maxima, Adam within 1e-6;
* probe slopes and their Jacobian from the batched 5-plane build against the
  oracle's IM and Jacobian of the probe maps (1e-5 / 1e-4 of the maxima);
* Gauss-Newton on the device: noise-free probe slopes (oracle, FP64) give back
  the misregistration; noisy slopes give the oracle's own Gauss-Newton fit.
"""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import im as oim, misreg as omr, mlp as omlp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(got, ref):
    return float(np.max(np.abs(np.asarray(got, np.float64) - ref)) / np.max(np.abs(ref)))


# ------------------------------------------------------------------ MLP
NET = dict(n_in=300, h1=96, h2=40, n_out=4, segments=((10, 50), (150, 70)))


def _net_and_params(S, seed=3):
    net = S.Mlp(NET["n_in"], NET["h1"], NET["h2"], NET["n_out"], NET["segments"])
    rng = np.random.default_rng(seed)
    sizes = [(96, 300), (96,), (40, 96), (40,), (4, 40), (4,)]
    parts = [rng.standard_normal(s) * (math.sqrt(2.0 / s[1]) if len(s) == 2 else 0.1)
             for s in sizes]
    packed = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
    assert packed.size == net.n_params
    P = [p.astype(np.float32).astype(np.float64) for p in parts]
    oparams = [(P[0], P[1]), (P[2], P[3]), (P[4], P[5])]
    return net, packed, oparams


def _full_input(xc):
    (s0, l0), (s1, l1) = NET["segments"]
    x = np.zeros((xc.shape[0], NET["n_in"]))
    x[:, s0:s0 + l0] = xc[:, :l0]
    x[:, s1:s1 + l1] = xc[:, l0:]
    return x


@pytest.mark.parametrize("B", [1, 5, 16, 17, 37, 256])
def test_mlp_forward_backward_parity(gpu_lib, B):
    import torch
    S = gpu_lib
    say(f"[case] mlp forward/backward B={B}")
    net, packed, oparams = _net_and_params(S)
    rng = np.random.default_rng(100 + B)
    xc = rng.standard_normal((B, 120)).astype(np.float32)
    t = rng.uniform(-1, 1, (B, 4)).astype(np.float32)
    dev = torch.device("cuda:0")
    params = torch.from_numpy(packed).to(dev)
    x = torch.from_numpy(xc).to(dev)
    tt = torch.from_numpy(t).to(dev)
    scratch = net.scratch(B, device=dev)
    y = net.forward(params, x, scratch)
    grads = torch.empty_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    net.backward(params, x, scratch, y, tt, grads, loss)
    torch.cuda.synchronize()
    yref, acts = omlp.forward(_full_input(xc.astype(np.float64)), oparams)
    assert rel_err(y.cpu().numpy(), yref) <= 1e-4
    assert abs(float(loss.item()) - omlp.mse(yref, t)) <= 1e-4 * omlp.mse(yref, t)
    gref = omlp.backward(acts, oparams, t.astype(np.float64))
    g = grads.cpu().numpy()
    for (lo, hi), ref in zip(net.layout(), [a for pair in gref for a in pair]):
        got = g[lo:hi].reshape(ref.shape)
        if np.max(np.abs(ref)) == 0:
            assert np.all(got == 0)
        else:
            assert rel_err(got, ref) <= 1e-4, (lo, hi)
    # W1 columns outside the two input segments carry exactly zero gradient
    W1 = g[net.layout()[0][0]:net.layout()[0][1]].reshape(96, 300)
    mask = np.ones(300, bool)
    mask[10:60] = False
    mask[150:220] = False
    assert np.all(W1[:, mask] == 0)


@pytest.mark.parametrize("B", [1, 37, 256, 1000])
def test_mlp_parity_estimator_shape(gpu_lib, B):
    """The estimator's own network, 2 x 4000 -> 512 -> 256 -> 4, fed the compact
    inputs of the learned-fit workload (20 probes x 52 subapertures per channel,
    2080 non-zero inputs of 8000), He-initialised as in training: forward and
    MSE backward against the FP64 oracle net on the zero-padded 8000 inputs."""
    import torch
    from paper_2606_07759_amd import learned
    S = gpu_lib
    say(f"[case] mlp estimator shape B={B}")
    nN = 20 * 52
    net = S.Mlp(8000, 512, 256, 4, ((0, nN), (4000, nN)))
    packed = learned.he_init(net, 12)
    rng = np.random.default_rng(200 + B)
    # non-zero biases, so their gradients and the ReLU masks are exercised
    for (lo, hi), is_bias in zip(net.layout(), (False, True) * 3):
        if is_bias:
            packed[lo:hi] = (0.05 * rng.standard_normal(hi - lo)).astype(np.float32)
    xc = rng.standard_normal((B, 2 * nN)).astype(np.float32)
    t = rng.uniform(-1, 1, (B, 4)).astype(np.float32)
    dev = torch.device("cuda:0")
    params = torch.from_numpy(packed).to(dev)
    scratch = net.scratch(B, device=dev)
    y = net.forward(params, torch.from_numpy(xc).to(dev), scratch)
    grads = torch.empty_like(params)
    net.backward(params, torch.from_numpy(xc).to(dev), scratch, y, torch.from_numpy(t).to(dev),
                 grads)
    torch.cuda.synchronize()
    lay = net.layout()
    shapes = [(512, 8000), (512,), (256, 512), (256,), (4, 256), (4,)]
    P = [packed[lo:hi].astype(np.float64).reshape(sh) for (lo, hi), sh in zip(lay, shapes)]
    oparams = [(P[0], P[1]), (P[2], P[3]), (P[4], P[5])]
    x = np.zeros((B, 8000))
    x[:, :nN] = xc[:, :nN]
    x[:, 4000:4000 + nN] = xc[:, nN:]
    yref, acts = omlp.forward(x, oparams)
    assert rel_err(y.cpu().numpy(), yref) <= 1e-4
    gref = omlp.backward(acts, oparams, t.astype(np.float64))
    g = grads.cpu().numpy()
    for (lo, hi), ref in zip(lay, [a for pair in gref for a in pair]):
        got = g[lo:hi].reshape(ref.shape)
        assert rel_err(got, ref) <= 1e-4, (lo, hi, rel_err(got, ref))


@pytest.mark.parametrize("B", [100, 333])
def test_mlp_parity_split_products(gpu_lib, B):
    """Layer widths and input lengths that are no multiples of the 64 x 64 GEMM
    tiles or the 32-wide K chunks, so that the products split K into ragged
    parts (the last one shorter) whose partial sums are reduced afterwards."""
    import torch
    from paper_2606_07759_amd import learned
    S = gpu_lib
    say(f"[case] mlp split products B={B}")
    segs = ((100, 350), (900, 351))
    net = S.Mlp(1500, 200, 70, 3, segs)
    packed = learned.he_init(net, 5)
    rng = np.random.default_rng(300 + B)
    for (lo, hi), is_bias in zip(net.layout(), (False, True) * 3):
        if is_bias:
            packed[lo:hi] = (0.05 * rng.standard_normal(hi - lo)).astype(np.float32)
    xc = rng.standard_normal((B, 701)).astype(np.float32)
    t = rng.uniform(-1, 1, (B, 3)).astype(np.float32)
    dev = torch.device("cuda:0")
    params = torch.from_numpy(packed).to(dev)
    scratch = net.scratch(B, device=dev)
    xd = torch.from_numpy(xc).to(dev)
    y = net.forward(params, xd, scratch)
    grads = torch.empty_like(params)
    net.backward(params, xd, scratch, y, torch.from_numpy(t).to(dev), grads)
    torch.cuda.synchronize()
    lay = net.layout()
    shapes = [(200, 1500), (200,), (70, 200), (70,), (3, 70), (3,)]
    P = [packed[lo:hi].astype(np.float64).reshape(sh) for (lo, hi), sh in zip(lay, shapes)]
    oparams = [(P[0], P[1]), (P[2], P[3]), (P[4], P[5])]
    x = np.zeros((B, 1500))
    x[:, 100:450] = xc[:, :350]
    x[:, 900:1251] = xc[:, 350:]
    yref, acts = omlp.forward(x, oparams)
    assert rel_err(y.cpu().numpy(), yref) <= 1e-4
    gref = omlp.backward(acts, oparams, t.astype(np.float64))
    g = grads.cpu().numpy()
    for (lo, hi), ref in zip(lay, [a for pair in gref for a in pair]):
        got = g[lo:hi].reshape(ref.shape)
        assert rel_err(got, ref) <= 1e-4, (lo, hi, rel_err(got, ref))
    # a second forward pass through the same scratch is bitwise the same
    y2 = net.forward(params, xd, scratch)
    assert torch.equal(y, y2)


def test_adam_step_parity(gpu_lib):
    import torch
    S = gpu_lib
    say("[case] adam")
    rng = np.random.default_rng(7)
    n = 10_007
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = (0.1 * rng.standard_normal(n)).astype(np.float32)
    v = np.abs(0.01 * rng.standard_normal(n)).astype(np.float32)
    dev = torch.device("cuda:0")
    tp, tg, tm, tv = (torch.from_numpy(a.copy()).to(dev) for a in (p, g, m, v))
    S.adam_step(tp, tg, tm, tv, step=3, lr=1e-3)
    torch.cuda.synchronize()
    rp, rm, rv = omlp.adam_step(p.astype(np.float64), g.astype(np.float64),
                                m.astype(np.float64), v.astype(np.float64), 3)
    assert np.max(np.abs(tp.cpu().numpy() - rp)) <= 1e-6 * np.max(np.abs(rp))
    assert rel_err(tm.cpu().numpy(), rm) <= 1e-6
    assert rel_err(tv.cpu().numpy(), rv) <= 1e-6


def test_mlp_training_reduces_loss(gpu_lib):
    """A few hundred Adam steps of the GPU kernels fit a smooth target map."""
    import torch
    S = gpu_lib
    say("[case] mlp training")
    net, packed, _ = _net_and_params(S, seed=5)
    rng = np.random.default_rng(9)
    n = 2048
    xc = rng.standard_normal((n, 120)).astype(np.float32)
    Wt = rng.standard_normal((120, 4)) / math.sqrt(120)
    t = np.tanh(xc @ Wt).astype(np.float32)
    dev = torch.device("cuda:0")
    params = torch.from_numpy(packed).to(dev)
    grads = torch.zeros_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    x = torch.from_numpy(xc).to(dev)
    tt = torch.from_numpy(t).to(dev)
    B = 128
    scratch = net.scratch(B, device=dev)
    out = torch.empty((B, 4), dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    first = last = None
    step = 0
    for ep in range(8):
        for k in range(n // B):
            xb = x[k * B:(k + 1) * B].contiguous()
            tb = tt[k * B:(k + 1) * B].contiguous()
            net.forward(params, xb, scratch, out)
            net.backward(params, xb, scratch, out, tb, grads, loss)
            step += 1
            S.adam_step(params, grads, m, v, step, lr=1e-3)
            if first is None:
                first = float(loss.item())
        last = float(loss.item())
    say(f"loss {first:.4f} -> {last:.4f}")
    assert last < 0.2 * first


# ------------------------------------------------------- misregistration
@pytest.fixture(scope="module")
def probe(gpu_lib):
    import torch
    S = gpu_lib
    pc = wl.probe_config()
    cfg = pc.scao
    wfs = S.Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid, device="cuda:0")
    maps = torch.from_numpy(pc.probe_maps).to("cuda:0")
    return pc, wfs, maps


THETAS = [
    (0.0, 0.0, 0.0, 1.0),
    (3.7, -6.2, math.radians(0.6), 1.013),
    (-9.5, 8.1, math.radians(-0.9), 0.982),
]


def test_misreg_slopes_and_jacobian_parity(gpu_lib, probe):
    import torch
    S = gpu_lib
    pc, wfs, maps = probe
    cfg = pc.scao
    say("[case] misreg slopes/jacobian")
    ctx = S.Misreg(wfs, maps, wl.LABEL_LO, wl.LABEL_HI, max_batch=4)
    th = torch.tensor(THETAS, dtype=torch.float64, device="cuda:0")
    s, J = ctx.slopes(th, jac=True)
    torch.cuda.synchronize()
    assert ctx.status() == 0
    s = s.cpu().numpy()
    J = J.cpu().numpy()
    F = pc.probe_maps.astype(np.float64)
    for i, theta in enumerate(THETAS):
        ref = omr.probe_slopes(F, theta, cfg.pupil, cfg.p, cfg.valid).ravel()
        assert rel_err(s[i], ref) <= 1e-5, i
        Jr = omr.probe_jacobian(F, theta, cfg.pupil, cfg.p, cfg.valid).reshape(4, -1)
        for j in range(4):
            assert rel_err(J[i, j], Jr[j]) <= 1e-4, (i, j)
    ctx.close()


@pytest.mark.parametrize("batched", [False, True], ids=["fused", "batched"])
def test_gn_recovers_noise_free(gpu_lib, probe, batched):
    import torch
    S = gpu_lib
    pc, wfs, maps = probe
    cfg = pc.scao
    say(f"[case] GN noise-free batched={batched}")
    truth = np.array(THETAS[1:] + [(1.2, 0.4, math.radians(0.2), 1.004)])
    F = pc.probe_maps.astype(np.float64)
    meas = np.stack([omr.probe_slopes(F, t, cfg.pupil, cfg.p, cfg.valid).ravel()
                     for t in truth]).astype(np.float32)
    ctx = S.Misreg(wfs, maps, wl.LABEL_LO, wl.LABEL_HI, max_batch=8, max_iter=30,
                   gn_batched=batched)
    for graph in (False, True):
        th, it = ctx.infer(torch.from_numpy(meas).cuda(), S.MISREG_GN, use_graph=graph)
        th = th.cpu().numpy()
        it = it.cpu().numpy()
        say("theta", th, "iters", it)
        assert np.all(np.abs(th[:, :2] - truth[:, :2]) <= 2e-3)
        assert np.all(np.abs(th[:, 2] - truth[:, 2]) <= 2e-5)
        assert np.all(np.abs(th[:, 3] - truth[:, 3]) <= 2e-5)
    assert ctx.status() == 0
    ctx.close()


@pytest.mark.parametrize("batched,n", [(False, 2), (False, 12), (True, 2)],
                         ids=["fused-multi", "fused-single", "batched"])
def test_gn_matches_oracle_on_noisy_slopes(gpu_lib, probe, batched, n):
    """n <= 8 samples split each sample over workgroups; more use one each."""
    import torch
    S = gpu_lib
    pc, wfs, maps = probe
    cfg = pc.scao
    say(f"[case] GN noisy vs oracle GN batched={batched} n={n}")
    F = pc.probe_maps.astype(np.float64)
    scale = 0.5 * (wl.LABEL_HI - wl.LABEL_LO)
    meas, refs = [], []
    for seed in range(1_000_000, 1_000_000 + n):
        theta, snr, rng = wl.draw_misreg_labels(seed)
        s = omr.probe_slopes(F, theta, cfg.pupil, cfg.p, cfg.valid).ravel()
        s = s + rng.standard_normal(s.size) * (np.sqrt(np.mean(s * s)) / snr)
        meas.append(s.astype(np.float32))
        ref, _, ok = omr.gauss_newton(meas[-1].astype(np.float64), F, cfg.pupil, cfg.p,
                                      cfg.valid, scale, max_iter=30)
        refs.append(ref)
    ctx = S.Misreg(wfs, maps, wl.LABEL_LO, wl.LABEL_HI, max_batch=n, max_iter=30,
                   gn_batched=batched)
    th, it = ctx.infer(torch.from_numpy(np.stack(meas)).cuda(), S.MISREG_GN)
    th = th.cpu().numpy()
    assert np.all(it.cpu().numpy() >= 1)   # -1 / -2 would flag a region or sync failure
    refs = np.array(refs)
    say("gpu", th, "oracle", refs)
    assert np.all(np.abs(th[:, :2] - refs[:, :2]) <= 5e-3)
    assert np.all(np.abs(th[:, 2] - refs[:, 2]) <= 5e-5)
    assert np.all(np.abs(th[:, 3] - refs[:, 3]) <= 5e-5)
    ctx.close()


def test_gn_large_grid_global_taps(gpu_lib):
    """A WFS whose probe footprint does not fit in LDS (12x12 subapertures of
    10 px, 4 smooth probe maps on 160^2): the one-launch Gauss-Newton reads its
    taps from global memory; noise-free slopes give back theta, noisy ones the
    oracle's fit."""
    import torch
    S = gpu_lib
    say("[case] GN large grid")
    pup = wl.pupil_mask(120, 120.0, 0.2)
    val = wl.valid_subapertures(pup, 10)
    c = (160 - 1) / 2.0
    yy, xx = np.mgrid[0:160, 0:160].astype(np.float64)
    maps = []
    for (ax, ay, sg) in ((0.0, 0.0, 30.0), (25.0, -10.0, 18.0), (-20.0, 22.0, 22.0), (5.0, 30.0, 15.0)):
        maps.append(np.exp(-((xx - c - ax) ** 2 + (yy - c - ay) ** 2) / (2 * sg * sg)))
    maps = np.stack(maps).astype(np.float32)
    F = maps.astype(np.float64)
    lo = np.array([-5.0, -5.0, math.radians(-1.0), 0.98])
    hi = np.array([5.0, 5.0, math.radians(1.0), 1.02])
    truth = np.array([(2.3, -1.7, math.radians(0.4), 1.008), (-4.1, 3.3, math.radians(-0.7), 0.985)])
    meas = np.stack([omr.probe_slopes(F, t, pup, 10, val).ravel() for t in truth]).astype(np.float32)
    wfs = S.Wfs.from_numpy(pup, 10, val, device="cuda:0")
    ctx = S.Misreg(wfs, torch.from_numpy(maps).cuda(), lo, hi, max_batch=2, max_iter=30)
    th, it = ctx.infer(torch.from_numpy(meas).cuda(), S.MISREG_GN)
    th = th.cpu().numpy()
    say("theta", th, "iters", it.cpu().numpy())
    assert np.all(np.abs(th[:, :2] - truth[:, :2]) <= 2e-3)
    assert np.all(np.abs(th[:, 2:] - truth[:, 2:]) <= 2e-5)
    ctx.close()
