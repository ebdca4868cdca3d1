"""Learned misregistration estimator: data synthesis, training and evaluation.

Everything that computes runs in the library's HIP kernels: probe slopes come
from the batched build (``Misreg.slopes``), the features from
``Misreg.features``, and the MLP is trained by the hand-written forward,
backward and Adam kernels.  torch provides device memory; numpy draws the
seeded labels and noise.

Readings of the learned-fit workload (the training recipe is not in the paper):
* probes: Noll Zernikes 2-21 fitted by the 9x9 DM, on the 8x8 SCAO WFS;
* labels: shift U(-1, 1) subaperture per axis, rotation U(-1, 1) deg,
  magnification U(0.98, 1.02), scaled to [-1, 1] for the network;
* noise: per-sample SNR U(20, 200), sigma = RMS(S(theta)) / SNR, i.i.d.
  Gaussian on every slope;
* inputs: 2 x feat_len (x and y slopes, probe-major, zero-padded), each
  feature standardised with the training-set mean and std;
* training: He-normal init (seeded), Adam (1e-3, 0.9, 0.999, 1e-8), batch 256,
  a 90/10 train/validation split, early stop on validation MSE.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Optional

import numpy as np

import workloads as wl

from . import MISREG_GN, MISREG_MLP, MISREG_MLP_GN, Misreg, Mlp, Wfs, adam_step


@dataclass
class ProbeSystem:
    wfs: Wfs
    probes: "object"        # torch [n_probe][128][128]
    lo: np.ndarray
    hi: np.ndarray
    n_probe: int
    n_valid: int

    @property
    def M(self) -> int:
        return self.n_probe * 2 * self.n_valid


def probe_system(device="cuda") -> ProbeSystem:
    import torch
    pc = wl.probe_config()
    cfg = pc.scao
    wfs = Wfs.from_numpy(cfg.pupil, cfg.p, cfg.valid, device=device)
    probes = torch.from_numpy(pc.probe_maps).to(device)
    return ProbeSystem(wfs, probes, wl.LABEL_LO.copy(), wl.LABEL_HI.copy(), len(pc.modes),
                       cfg.n_valid)


def draw(seeds, M: int):
    """Labels theta [n][4], SNRs [n] and unit-normal noise [n][M] per seed."""
    th = np.empty((len(seeds), 4))
    snr = np.empty(len(seeds))
    noise = np.empty((len(seeds), M), dtype=np.float32)
    for i, s in enumerate(seeds):
        t, r, rng = wl.draw_misreg_labels(int(s))
        th[i] = t
        snr[i] = r
        noise[i] = rng.standard_normal(M)
    return th, snr, noise


def synthesize(ctx: Misreg, theta, snr, noise, batch: int):
    """Noisy probe slopes [n][M] (GPU float32) for the given labels."""
    import torch
    dev = ctx.probes.device
    n = theta.shape[0]
    out = torch.empty((n, ctx.M), dtype=torch.float32, device=dev)
    th = torch.from_numpy(theta).to(dev)
    nz = torch.from_numpy(noise).to(dev)
    sn = torch.from_numpy(snr).to(dev).float()
    for a in range(0, n, batch):
        b = min(n, a + batch)
        s = ctx.slopes(th[a:b].contiguous())
        rms = torch.sqrt((s * s).mean(dim=1, keepdim=True))
        out[a:b] = s + nz[a:b] * (rms / sn[a:b, None])
    return out


def net_for(system: ProbeSystem, feat_len: int = 4000, h1: int = 512, h2: int = 256) -> Mlp:
    nN = system.n_probe * system.n_valid
    return Mlp(2 * feat_len, h1, h2, 4, ((0, nN), (feat_len, nN)))


def he_init(net: Mlp, seed: int):
    """He-normal weights, zero biases, packed (float32, host)."""
    rng = wl.rng_for(seed)
    d = net.desc
    shapes = [(d.h1, d.n_in), (d.h1,), (d.h2, d.h1), (d.h2,), (d.n_out, d.h2), (d.n_out,)]
    parts = []
    for sh in shapes:
        if len(sh) == 2:
            parts.append(rng.standard_normal(sh).ravel() * math.sqrt(2.0 / sh[1]))
        else:
            parts.append(np.zeros(sh))
    return np.concatenate(parts).astype(np.float32)


@dataclass
class Trained:
    net: Mlp
    params: "object"
    mean: "object"
    std: "object"
    feat_len: int
    history: list
    seconds: float


def train(system: ProbeSystem, slopes, theta, *, feat_len=4000, epochs=60, batch=256, lr=1e-3,
          lr_min=1e-5, seed=0, val_frac=0.1, patience=12, log=None,
          checkpoint: Optional[str] = None, resume: Optional[str] = None,
          stop_after: Optional[int] = None) -> Trained:
    """Train the estimator on (noisy slopes [n][M] GPU, theta [n][4] numpy).

    Adam with a cosine learning-rate decay from ``lr`` to ``lr_min`` over the
    epochs; the parameters with the best validation MSE are kept.

    ``checkpoint``: a ``.npz`` path written after every epoch with the
    parameters, the Adam moments and step, the best parameters so far, the
    early-stop state, the history and the state of the shuffling generator.
    ``resume``: such a file; training continues after its last epoch, and with
    the same data and settings ends where an uninterrupted run would (the
    kernels reduce in a fixed order).  ``stop_after``: leave after that many
    epochs of this call (an interrupted run, for tests)."""
    import torch
    dev = slopes.device
    net = net_for(system, feat_len)
    ctx = Misreg(system.wfs, system.probes, system.lo, system.hi, max_batch=1)
    raw = ctx.features(slopes)                      # compact features, unstandardised
    n = raw.shape[0]
    n_val = max(1, int(round(val_frac * n)))
    n_tr = n - n_val
    mean = raw[:n_tr].mean(dim=0)
    std = raw[:n_tr].std(dim=0).clamp_min(1e-12)
    x = ctx.features(slopes, mean.contiguous(), std.contiguous())
    ctx.close()
    lo = torch.from_numpy(system.lo).to(dev)
    hi = torch.from_numpy(system.hi).to(dev)
    y = ((torch.from_numpy(theta).to(dev) - lo) / (hi - lo) * 2 - 1).float().contiguous()
    params = torch.from_numpy(he_init(net, seed)).to(dev)
    grads = torch.zeros_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    scratch = net.scratch(batch, device=dev)
    vscratch = net.scratch(n_val, device=dev)
    out = torch.empty((batch, 4), dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    g = torch.Generator(device="cpu").manual_seed(seed)
    best, best_params, bad, step, hist = float("inf"), params.clone(), 0, 0, []
    ep0 = 0
    if resume is not None:
        with np.load(resume, allow_pickle=False) as z:
            if int(z["n_params"]) != params.numel():
                raise ValueError("checkpoint is for another network")
            params.copy_(torch.from_numpy(z["params"]))
            m.copy_(torch.from_numpy(z["m"]))
            v.copy_(torch.from_numpy(z["v"]))
            best_params = torch.from_numpy(z["best_params"]).to(dev)
            best, bad, step = float(z["best"]), int(z["bad"]), int(z["step"])
            hist = [tuple(r) for r in z["history"].tolist()]
            ep0 = int(z["epoch"]) + 1
            g.set_state(torch.from_numpy(z["rng_state"]))
    t0 = time.perf_counter()
    done = 0
    for ep in range(ep0, epochs):
        if stop_after is not None and done >= stop_after:
            break
        done += 1
        perm = torch.randperm(n_tr, generator=g).to(dev)
        tot = 0.0
        nb = n_tr // batch
        for k in range(nb):
            idx = perm[k * batch:(k + 1) * batch]
            xb = x[idx].contiguous()
            yb = y[idx].contiguous()
            net.forward(params, xb, scratch, out)
            net.backward(params, xb, scratch, out, yb, grads, loss)
            step += 1
            t = step / float(max(1, epochs * nb))
            adam_step(params, grads, m, v, step,
                      lr=lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * min(1.0, t))))
            tot += float(loss.item()) if k == nb - 1 else 0.0
        yv = net.forward(params, x[n_tr:].contiguous(), vscratch)
        vl = float(((yv - y[n_tr:]) ** 2).mean().item())
        hist.append((ep, tot, vl))
        if log:
            log(f"epoch {ep}: train(last batch) {tot:.5f} val {vl:.5f}")
        if vl < best:
            best, best_params, bad = vl, params.clone(), 0
        else:
            bad += 1
        if checkpoint is not None:
            np.savez(checkpoint, params=params.cpu().numpy(), m=m.cpu().numpy(),
                     v=v.cpu().numpy(), best_params=best_params.cpu().numpy(),
                     best=np.float64(best), bad=np.int64(bad), step=np.int64(step),
                     epoch=np.int64(ep), history=np.array(hist, dtype=np.float64).reshape(-1, 3),
                     rng_state=g.get_state().numpy(), n_params=np.int64(params.numel()))
        if bad >= patience:
            break
    torch.cuda.synchronize()
    return Trained(net, best_params, mean.contiguous(), std.contiguous(), feat_len, hist,
                   time.perf_counter() - t0)


def save_trained(path: str, trained: Trained) -> None:
    """The trained estimator (network shape, parameters, feature mean and std)
    as a ``.npz`` file."""
    d = trained.net.desc
    np.savez(path, params=trained.params.cpu().numpy(), mean=trained.mean.cpu().numpy(),
             std=trained.std.cpu().numpy(), feat_len=np.int64(trained.feat_len),
             shape=np.array([d.n_in, d.h1, d.h2, d.n_out, d.seg0, d.len0, d.seg1, d.len1],
                            dtype=np.int64),
             history=np.array(trained.history, dtype=np.float64).reshape(-1, 3),
             seconds=np.float64(trained.seconds))


def load_trained(path: str, device="cuda") -> Trained:
    """A trained estimator saved by :func:`save_trained`, on ``device``."""
    import torch
    with np.load(path, allow_pickle=False) as z:
        n_in, h1, h2, n_out, s0, l0, s1, l1 = (int(x) for x in z["shape"])
        net = Mlp(n_in, h1, h2, n_out, ((s0, l0), (s1, l1)))
        params = torch.from_numpy(z["params"]).to(device)
        if params.numel() != net.n_params:
            raise ValueError("parameter count does not match the network shape")
        return Trained(net, params, torch.from_numpy(z["mean"]).to(device),
                       torch.from_numpy(z["std"]).to(device), int(z["feat_len"]),
                       [tuple(r) for r in z["history"].tolist()], float(z["seconds"]))


def estimator(system: ProbeSystem, trained: Optional[Trained], max_batch: int,
              max_iter: int = 20) -> Misreg:
    mlp = None
    if trained is not None:
        mlp = (trained.net, trained.params, trained.mean, trained.std, trained.feat_len)
    return Misreg(system.wfs, system.probes, system.lo, system.hi, max_batch=max_batch,
                  max_iter=max_iter, mlp=mlp)


def time_fit(ctx: Misreg, slopes, mode, reps=20, iter_cap=0):
    """Median and p95 wall time (ms) of one fit call on the GPU (graph replay)."""
    import torch
    B = slopes.shape[0]
    out = (torch.empty((B, 4), dtype=torch.float64, device=slopes.device),
           torch.empty(B, dtype=torch.int32, device=slopes.device))
    ctx.infer(slopes, mode, iter_cap=iter_cap, out=out)   # capture
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.infer(slopes, mode, iter_cap=iter_cap, out=out)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    ts = np.sort(np.array(ts))
    return float(np.median(ts)), float(ts[int(0.95 * (len(ts) - 1))])


def evaluate(system: ProbeSystem, trained: Trained, seeds, batch: int = 1000,
             max_iter: int = 20, timing_reps: int = 20) -> dict:
    """Learned estimate against the Gauss-Newton fit on held-out seeds.

    Every seed gives one noisy probe-slope sample (labels, SNR and noise drawn
    from the seed).  Reported, per axis, in subapertures (shift / p) and as
    pupil-edge displacement for rotation (rho * R) and magnification
    ((m - 1) * R), R = pupil radius in subapertures:
      * RMS of the MLP estimate minus the GN estimate (GN from theta0);
      * RMS of each estimate minus the truth;
      * GN iterations from theta0 and from the MLP estimate;
      * median / p95 latency of one fit call at batch 1 and at ``batch``.
    """
    import torch
    dev = system.probes.device
    seeds = np.asarray(seeds)
    n = len(seeds)
    theta, snr, noise = draw(seeds, system.M)
    gen = Misreg(system.wfs, system.probes, system.lo, system.hi, max_batch=batch)
    slopes = synthesize(gen, theta, snr, noise, batch)
    gen.close()
    est = estimator(system, trained, max_batch=batch, max_iter=max_iter)
    res = {MISREG_GN: [], MISREG_MLP: [], MISREG_MLP_GN: []}
    its = {MISREG_GN: [], MISREG_MLP_GN: []}
    unconv = {MISREG_GN: 0, MISREG_MLP_GN: 0}
    for a in range(0, n, batch):
        b = min(n, a + batch)
        s = slopes[a:b].contiguous()
        for mode in (MISREG_GN, MISREG_MLP, MISREG_MLP_GN):
            th, it = est.infer(s, mode, use_graph=False)
            res[mode].append(th.cpu().numpy())
            if mode in its:
                its[mode].append(it.cpu().numpy())
                unconv[mode] += est.unconverged()
    for k in res:
        res[k] = np.concatenate(res[k])
    for k in its:
        its[k] = np.concatenate(its[k])
    p = float(system.wfs.p)
    radius = 0.5 * system.wfs.n_sub_x                     # pupil radius in subapertures
    unit = np.array([1.0 / p, 1.0 / p, radius, radius])  # -> subapertures
    shift = np.array([0.0, 0.0, 0.0, 1.0])

    def rms(x, y):
        d = ((x - shift) - (y - shift)) * unit
        return [float(v) for v in np.sqrt(np.mean(d * d, axis=0))]

    out = {
        "n_samples": int(n),
        "units": "subapertures (shift/p; rot*R; (mag-1)*R with R the pupil radius in subapertures)",
        "rms_mlp_vs_gn": rms(res[MISREG_MLP], res[MISREG_GN]),
        "rms_mlp_gn_vs_gn": rms(res[MISREG_MLP_GN], res[MISREG_GN]),
        "rms_gn_vs_truth": rms(res[MISREG_GN], theta),
        "rms_mlp_vs_truth": rms(res[MISREG_MLP], theta),
        "gn_iters_mean": float(its[MISREG_GN].mean()),
        "gn_iters_max": int(its[MISREG_GN].max()),
        "mlp_gn_iters_mean": float(its[MISREG_MLP_GN].mean()),
        "mlp_gn_iters_max": int(its[MISREG_MLP_GN].max()),
        "gn_unconverged": int(unconv[MISREG_GN]),
        "mlp_gn_unconverged": int(unconv[MISREG_MLP_GN]),
        "gn_capped_seeds": [int(v) for v in seeds[its[MISREG_GN] >= max_iter]],
    }
    timing = {}
    for bsz in (1, min(batch, n)):
        s = slopes[:bsz].contiguous()
        for mode, name in ((MISREG_GN, "gn"), (MISREG_MLP, "mlp"), (MISREG_MLP_GN, "mlp_gn")):
            med, p95 = time_fit(est, s, mode, reps=timing_reps)
            timing[f"{name}_b{bsz}_ms"] = [med, p95]
    out["latency_ms_median_p95"] = timing
    est.close()
    torch.cuda.synchronize(dev)
    return out


def run(n_train: int = 50_000, n_eval: int = 1000, epochs: int = 60, seed: int = 0,
        log=None) -> dict:
    """The whole learned-fit workload: synthesise the training set with the
    library, train on the GPU kernels, evaluate on held-out seeds."""
    import torch
    t0 = time.perf_counter()
    system = probe_system("cuda")
    theta, snr, noise = draw(np.arange(n_train), system.M)
    gen = Misreg(system.wfs, system.probes, system.lo, system.hi, max_batch=1000)
    slopes = synthesize(gen, theta, snr, noise, 1000)
    gen.close()
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    trained = train(system, slopes, theta, epochs=epochs, seed=seed, log=log)
    rep = evaluate(system, trained, np.arange(1_000_000, 1_000_000 + n_eval))
    rep.update({"n_train": n_train, "epochs_run": len(trained.history),
                "train_seconds": trained.seconds, "data_seconds": t_data,
                "final_val_mse": trained.history[-1][2] if trained.history else None})
    return rep


__all__ = ["ProbeSystem", "probe_system", "draw", "synthesize", "net_for", "he_init", "train",
           "estimator", "time_fit", "evaluate", "run", "MISREG_GN", "MISREG_MLP", "MISREG_MLP_GN"]


def replay_fits(reps: int = 3):
    """Three graph replays of each estimate mode (GN, MLP, MLP->GN) on one
    held-out sample, with an untrained (He-initialised) network: the
    workload a kernel trace of the fit is taken on."""
    import torch
    system = probe_system("cuda")
    theta, snr, noise = draw(np.arange(1_000_000, 1_000_001), system.M)
    gen = Misreg(system.wfs, system.probes, system.lo, system.hi, max_batch=1)
    slopes = synthesize(gen, theta, snr, noise, 1)
    gen.close()
    net = net_for(system)
    params = torch.from_numpy(he_init(net, 0)).cuda()
    mean = torch.zeros(system.M, device="cuda")
    std = torch.ones(system.M, device="cuda")
    ctx = Misreg(system.wfs, system.probes, system.lo, system.hi, max_batch=1, max_iter=20,
                 mlp=(net, params, mean, std, 4000))
    out = (torch.empty((1, 4), dtype=torch.float64, device="cuda"),
           torch.empty(1, dtype=torch.int32, device="cuda"))
    for mode in (MISREG_GN, MISREG_MLP, MISREG_MLP_GN):
        for _ in range(reps):
            ctx.infer(slopes, mode, use_graph=True, out=out)
        torch.cuda.synchronize()
        print("mode", mode, "iters", out[1].cpu().numpy(), flush=True)
    ctx.close()


if __name__ == "__main__":
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="train and evaluate the learned misregistration estimator")
    ap.add_argument("--n-train", type=int, default=50_000)
    ap.add_argument("--n-eval", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--replay-fits", action="store_true",
                    help="only replay the three estimate modes (for a kernel trace)")
    args = ap.parse_args()
    if args.replay_fits:
        replay_fits()
        sys.exit(0)
    rep = run(args.n_train, args.n_eval, args.epochs,
              log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(rep), flush=True)
