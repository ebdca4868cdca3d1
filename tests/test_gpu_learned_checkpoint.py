"""Checkpoints of the estimator's training and of the trained estimator.

A short training run (2000 library-generated samples, a small network) is
made three ways: uninterrupted for 6 epochs; 3 epochs with a per-epoch
checkpoint, then resumed from it for the rest.  The resumed run must end with
bitwise the same parameters, Adam state and history (the kernels reduce in a
fixed order and the shuffling generator's state is in the checkpoint).  A
trained estimator saved and loaded must give bitwise the same estimates.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_training_resume_and_saved_estimator(gpu_lib, tmp_path):
    import torch
    from paper_2606_07759_amd import learned
    say("[case] training checkpoint: synthesising 2000 samples")
    system = learned.probe_system("cuda:0")
    n = 2000
    theta, snr, noise = learned.draw(np.arange(n), system.M)
    gen = gpu_lib.Misreg(system.wfs, system.probes, system.lo, system.hi, max_batch=1000)
    slopes = learned.synthesize(gen, theta, snr, noise, 1000)
    gen.close()
    kw = dict(feat_len=1200, epochs=6, batch=128, patience=100, seed=3)
    full = learned.train(system, slopes, theta, **kw)
    ck = str(tmp_path / "train.npz")
    part = learned.train(system, slopes, theta, checkpoint=ck, stop_after=3, **kw)
    assert len(part.history) == 3
    with np.load(ck) as z:
        assert int(z["epoch"]) == 2 and int(z["step"]) > 0
    rest = learned.train(system, slopes, theta, resume=ck, checkpoint=ck, **kw)
    say(f"full {len(full.history)} epochs, resumed {len(rest.history)}")
    assert len(rest.history) == len(full.history) == 6
    assert np.array_equal(np.array(rest.history), np.array(full.history))
    assert torch.equal(rest.params, full.params)
    with np.load(ck) as z:
        assert int(z["epoch"]) == 5
    # the trained estimator, saved and loaded
    path = str(tmp_path / "estimator.npz")
    learned.save_trained(path, full)
    back = learned.load_trained(path, "cuda:0")
    assert back.feat_len == full.feat_len and torch.equal(back.params, full.params)
    assert torch.equal(back.mean, full.mean) and torch.equal(back.std, full.std)
    seeds = np.arange(5_000_000, 5_000_064)
    th, sn, no = learned.draw(seeds, system.M)
    est = [learned.estimator(system, t, 64) for t in (full, back)]
    s = learned.synthesize(est[0], th, sn, no, 64)
    outs = []
    for e in est:
        theta_hat, _ = e.infer(s, gpu_lib.MISREG_MLP)
        outs.append(theta_hat.clone())
        e.close()
    assert torch.equal(outs[0], outs[1])
