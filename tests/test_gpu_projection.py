"""GPU parity of the tomographic projection (paper Sec. 2.5) against the FP64
oracle, through the C ABI.

* the FP64 MFMA GEMM on ragged sizes in both operand layouts, with alpha and
  beta, in both tile shapes, against numpy's FP64 product (1e-12 of the
  result's maximum);
* the blocked Cholesky (lower factor against numpy's) and the two blocked
  triangular solves on a ragged SPD system (1e-10), and the not-positive-
  definite flag;
* the sampled projection matrices (footprint shifts per direction, 1x1 and 2x2
  binning) against the oracle's (1e-12);
* P_opt of a two-DM, two-layer system over three directions against the
  oracle's plain solve (1e-9 of its maximum).
"""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import projection as opj

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_gemm_f64_layouts(gpu_lib):
    S = gpu_lib
    rng = np.random.default_rng(1)
    for M, N, K in ((100, 70, 37), (64, 64, 16), (1, 130, 5), (129, 3, 200), (70, 33, 48)):
        say(f"[case] gemm {M}x{N}x{K}")
        Xk = rng.standard_normal((K, M))          # X(k, m) = Xk[k, m]: sxk = M, sxm = 1
        Yk = rng.standard_normal((N, K))          # Y(k, n) = Yk[n, k]: syk = 1, syn = K
        C0 = rng.standard_normal((M, N))
        Cd = dev(C0)
        S.gemm_f64(M, N, K, -0.5, dev(Xk), M, 1, dev(Yk), 1, K, 0.3, Cd, N)
        ref = -0.5 * Xk.T @ Yk.T + 0.3 * C0
        assert np.max(np.abs(Cd.cpu().numpy() - ref)) <= 1e-12 * np.abs(ref).max()


def test_gemm_f64_large_tiles(gpu_lib):
    """Products large enough for the 256 x 128 tile shape (at least 256 such
    tiles), ragged in m, n and k, in both operand layouts."""
    S = gpu_lib
    rng = np.random.default_rng(11)
    for M, N, K, k_unit in ((4100, 2060, 301, True), (4097, 2049, 37, False)):
        say(f"[case] gemm large {M}x{N}x{K} k-unit-stride={k_unit}")
        if k_unit:
            Xm = rng.standard_normal((M, K))      # X(k, m) = Xm[m, k]: sxk = 1, sxm = K
            Yn = rng.standard_normal((N, K))      # Y(k, n) = Yn[n, k]: syk = 1, syn = K
            Cd = dev(np.zeros((M, N)))
            S.gemm_f64(M, N, K, 1.0, dev(Xm), 1, K, dev(Yn), 1, K, 0.0, Cd, N)
            ref = Xm @ Yn.T
        else:
            Xk = rng.standard_normal((K, M))      # sxk = M, sxm = 1
            Yk = rng.standard_normal((K, N))      # syk = N, syn = 1
            C0 = rng.standard_normal((M, N))
            Cd = dev(C0)
            S.gemm_f64(M, N, K, 0.75, dev(Xk), M, 1, dev(Yk), N, 1, -1.25, Cd, N)
            ref = 0.75 * Xk.T @ Yk - 1.25 * C0
        assert np.max(np.abs(Cd.cpu().numpy() - ref)) <= 1e-12 * np.abs(ref).max()


def test_cholesky_large_trailing_updates(gpu_lib):
    """A Cholesky factor large enough that its trailing lower-triangle updates
    run in the 256 x 128 tile shape (tiles wholly above the diagonal skipped)."""
    import torch
    S = gpu_lib
    rng = np.random.default_rng(12)
    n = 4100
    R = rng.standard_normal((n, 64))
    A = R @ R.T + n * np.eye(n)
    say("[case] potrf large", n)
    Ad = dev(A)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    S.potrf_f64(Ad, st)
    assert int(st.item()) == 0
    L = np.tril(Ad.cpu().numpy())
    Lref = np.linalg.cholesky(A)
    assert np.max(np.abs(L - Lref)) <= 1e-12 * np.abs(Lref).max()


def test_cholesky_and_solves(gpu_lib):
    import torch
    S = gpu_lib
    rng = np.random.default_rng(2)
    n, m = 150, 33
    R = rng.standard_normal((n, n))
    A = R.T @ R + n * np.eye(n)
    B = rng.standard_normal((n, m))
    say("[case] potrf/potrs", n, m)
    Ad = dev(A)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    S.potrf_f64(Ad, st)
    L = np.tril(Ad.cpu().numpy())
    assert int(st.item()) == 0
    Lref = np.linalg.cholesky(A)
    assert np.max(np.abs(L - Lref)) <= 1e-12 * np.abs(Lref).max()
    Bd = dev(B)
    S.potrs_f64(Ad, Bd)
    X = np.linalg.solve(A, B)
    assert np.max(np.abs(Bd.cpu().numpy() - X)) <= 1e-10 * np.abs(X).max()
    # an indefinite matrix is flagged
    D = np.diag(np.r_[np.ones(70), -np.ones(10)])
    st.zero_()
    S.potrf_f64(dev(D), st)
    assert int(st.item()) == 1


def system():
    """Two DMs (ground and 6 km) and two layers (3 km, 9 km) of Gaussian bases,
    a 48-px pupil at 0.5 m per pixel, three directions (on axis, +-30 arcsec)."""
    g0 = wl.actuator_grid(9, 6.0, 56)
    g1 = wl.actuator_grid(7, 9.0, 64)
    l0 = wl.actuator_grid(8, 8.0, 64)
    l1 = wl.actuator_grid(6, 12.0, 72)
    dms = [(wl.if_stack(g0), 0.0, 0.5), (wl.if_stack(g1), 6000.0, 0.5)]
    layers = [(wl.if_stack(l0), 3000.0, 0.5), (wl.if_stack(l1), 9000.0, 0.5)]
    a = math.radians(30.0 / 3600.0)
    dirs = np.array([[0.0, 0.0], [a, -0.5 * a], [-0.7 * a, a]])
    pupil = wl.pupil_mask(48, 48.0, 0.14)
    return dms, layers, dirs, pupil


@pytest.mark.parametrize("b", [1, 2])
def test_projection_matrix_parity(gpu_lib, b):
    S = gpu_lib
    dms, layers, dirs, pupil = system()
    say(f"[case] projection matrix bin {b}")
    comps = dms + layers
    Pt = S.proj_matrix([(dev(F), h, s) for F, h, s in comps], dirs, pupil, 0.5, bin=b)
    ref = opj.projection_matrix(comps, dirs, pupil, 0.5, b)
    got = Pt.cpu().numpy().T
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.abs(ref).max()


def system_many_blocks():
    """The same geometry with denser DMs: 586 DM bases, so the Cholesky and the
    solves run over 9 diagonal blocks of 64 and a ragged last one."""
    dms, layers, dirs, pupil = system()
    g0 = wl.actuator_grid(19, 3.0, 56)
    g1 = wl.actuator_grid(15, 4.3, 64)
    dms = [(wl.if_stack(g0), 0.0, 0.5), (wl.if_stack(g1), 6000.0, 0.5)]
    return dms, layers, dirs, pupil


@pytest.mark.parametrize("many", [False, True])
def test_popt_parity(gpu_lib, many):
    S = gpu_lib
    dms, layers, dirs, pupil = system_many_blocks() if many else system()
    say(f"[case] P_opt, {sum(F.shape[0] for F, _, _ in dms)} DM bases")
    P_dm = opj.projection_matrix(dms, dirs, pupil, 0.5, 1)
    P_l = opj.projection_matrix(layers, dirs, pupil, 0.5, 1)
    lam = 1e-3 * np.trace(P_dm.T @ P_dm) / P_dm.shape[1]
    ref = opj.p_opt(P_dm, P_l, lam)
    got = S.proj_opt([(dev(F), h, s) for F, h, s in dms], [(dev(F), h, s) for F, h, s in layers],
                     dirs, pupil, 0.5, lam).cpu().numpy()
    e = np.max(np.abs(got - ref)) / np.abs(ref).max()
    say(f"  P_opt {got.shape}: rel err {e:.2e}")
    assert e <= 1e-9
