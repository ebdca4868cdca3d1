"""Python binding of the MI355X synthetic interaction-matrix library.

Argument marshalling only: every step of the interaction-matrix path runs in the
HIP kernels of ``libsynim.so`` (C ABI in ``include/synim.h``).  PyTorch supplies
device memory and the current stream.  There is no CPU fallback: if the
library is missing or no GPU is present, the calls raise.

Geometry conventions (pixel centres, inverse map, IM layout) are those of the
C header.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

from . import _abi

_LIB: Optional[C.CDLL] = None

STATUS_OOB = -4              # SYNIM_E_OOB
STATUS_NOT_CONVERGED = -7    # SYNIM_E_NOT_CONVERGED


class SynimError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _LIB.synim_status_str(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{where}: {msg} ({status})")


def load() -> C.CDLL:
    """Load ``libsynim.so`` (once); raises if it is not built."""
    global _LIB
    if _LIB is None:
        _LIB = _abi.load_library()
    return _LIB


def _check(rc: int, where: str):
    if rc != 0:
        raise SynimError(rc, where)


def _torch():
    import torch
    return torch


def _stream_handle(device) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


def _dev_f32(t, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    return t


# ------------------------------------------------------------------- geometry
def _affine_struct(A) -> _abi.SynimAffine:
    if isinstance(A, _abi.SynimAffine):
        return A
    M = np.asarray(A, dtype=np.float64).reshape(2, 3)
    s = _abi.SynimAffine()
    for i in range(2):
        for j in range(2):
            s.A[i][j] = M[i, j]
        s.b[i] = M[i, 2]
    return s


def affine_to_array(s: _abi.SynimAffine) -> np.ndarray:
    return np.array([[s.A[0][0], s.A[0][1], s.b[0]], [s.A[1][0], s.A[1][1], s.b[1]]])


def affine_from_misreg(theta: Sequence[float], H_in: int, W_in: int, H_out: int, W_out: int,
                       kappa: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """(A [2x3], dA [4x2x3]) of p_s = A[:, :2] p_o + A[:, 2] and its derivative maps."""
    lib = load()
    th = _abi.SynimMisreg(*[float(v) for v in theta])
    A = _abi.SynimAffine()
    dA = (_abi.SynimAffine * 4)()
    _check(lib.synim_affine_from_misreg(C.byref(th), H_in, W_in, H_out, W_out, float(kappa),
                                        C.byref(A), dA), "affine_from_misreg")
    return affine_to_array(A), np.stack([affine_to_array(dA[j]) for j in range(4)])


def affine_from_geometry(g, H_in: int, W_in: int, H_out: int, W_out: int) -> np.ndarray:
    """Inverse map [2x3] of a composite geometry (fields as ``synim_geometry``)."""
    lib = load()
    s = _abi.SynimGeometry(**{n: float(getattr(g, n)) for n, _ in _abi.SynimGeometry._fields_})
    A = _abi.SynimAffine()
    _check(lib.synim_affine_from_geometry(C.byref(s), H_in, W_in, H_out, W_out, C.byref(A)),
           "affine_from_geometry")
    return affine_to_array(A)


# ------------------------------------------------------------------------ WFS
@dataclass
class Wfs:
    """Device-resident Shack-Hartmann WFS description (pupil and valid list)."""
    n_sub_x: int
    n_sub_y: int
    p: int
    valid: "object"    # torch int32 [N] on the GPU, ascending
    pupil: "object"    # torch uint8 [n_sub_y*p][n_sub_x*p] on the GPU

    @classmethod
    def from_numpy(cls, pupil: np.ndarray, p: int, valid: np.ndarray, device="cuda"):
        torch = _torch()
        H, W = pupil.shape
        return cls(W // p, H // p, p,
                   torch.from_numpy(np.ascontiguousarray(valid, dtype=np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(pupil, dtype=np.uint8)).to(device))

    @property
    def n_valid(self) -> int:
        return int(self.valid.numel())

    @property
    def shape(self) -> Tuple[int, int]:
        return self.n_sub_y * self.p, self.n_sub_x * self.p

    def struct(self) -> _abi.SynimWfs:
        return _abi.SynimWfs(self.n_sub_x, self.n_sub_y, self.p, self.n_valid,
                             self.valid.data_ptr(), self.pupil.data_ptr())


# ---------------------------------------------------------- standalone steps
def affine_warp(ifs, A, H_out: int, W_out: int, halo: int = 1, out=None, oob=None):
    """Bilinear resampling of ifs [n][H_in][W_in] -> [n][H_out+2h][W_out+2h]."""
    torch = _torch()
    lib = load()
    _dev_f32(ifs, "ifs")
    n, H_in, W_in = ifs.shape
    if out is None:
        out = torch.empty((n, H_out + 2 * halo, W_out + 2 * halo), dtype=torch.float32,
                          device=ifs.device)
    a = _affine_struct(A)
    _check(lib.synim_affine_warp(ifs.data_ptr(), n, H_in, W_in, C.byref(a), H_out, W_out, halo,
                                 out.data_ptr(), oob.data_ptr() if oob is not None else None,
                                 _stream_handle(ifs.device)), "affine_warp")
    return out


def sa_slopes(phase, wfs: Wfs, out=None):
    """Slopes [n][2N] of haloed phase maps [n][H+2][W+2]."""
    torch = _torch()
    lib = load()
    _dev_f32(phase, "phase")
    n = phase.shape[0]
    H, W = wfs.shape
    if tuple(phase.shape[1:]) != (H + 2, W + 2):
        raise ValueError("phase must be [n][H+2][W+2]")
    if out is None:
        out = torch.empty((n, 2 * wfs.n_valid), dtype=torch.float32, device=phase.device)
    s = wfs.struct()
    _check(lib.synim_sa_slopes(phase.data_ptr(), n, C.byref(s), out.data_ptr(),
                               _stream_handle(phase.device)), "sa_slopes")
    return out


# ------------------------------------------------------------------ fused path
def im_workspace_bytes(wfs: Wfs, A, planes: int = 1) -> int:
    lib = load()
    s = wfs.struct()
    a = _affine_struct(A)
    n = C.c_size_t(0)
    _check(lib.synim_im_workspace(C.byref(s), C.byref(a), planes, C.byref(n)), "im_workspace")
    return int(n.value)


def _workspace(wfs, A, planes, ws, device):
    torch = _torch()
    need = im_workspace_bytes(wfs, A, planes)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
    return ws


def im_build(ifs, A, wfs: Wfs, out=None, ws=None):
    """IM [n_act][2N] (actuator-major) of ifs [n_act][H_in][W_in]."""
    torch = _torch()
    lib = load()
    _dev_f32(ifs, "ifs")
    n, H_in, W_in = ifs.shape
    if out is None:
        out = torch.empty((n, 2 * wfs.n_valid), dtype=torch.float32, device=ifs.device)
    ws = _workspace(wfs, A, 1, ws, ifs.device)
    s = wfs.struct()
    a = _affine_struct(A)
    _check(lib.synim_im_build(ifs.data_ptr(), n, H_in, W_in, C.byref(a), C.byref(s),
                              out.data_ptr(), ws.data_ptr(), ws.numel(),
                              _stream_handle(ifs.device)), "im_build")
    return out


def im_build_tsum(ifs, A, wfs: Wfs, out=None, ws=None):
    """IM with the telescoping-sum (G-tilt) slope engine (``synim_im_build_tsum``)."""
    torch = _torch()
    lib = load()
    _dev_f32(ifs, "ifs")
    n, H_in, W_in = ifs.shape
    if out is None:
        out = torch.empty((n, 2 * wfs.n_valid), dtype=torch.float32, device=ifs.device)
    ws = _workspace(wfs, A, 1, ws, ifs.device)
    s = wfs.struct()
    a = _affine_struct(A)
    _check(lib.synim_im_build_tsum(ifs.data_ptr(), n, H_in, W_in, C.byref(a), C.byref(s),
                                   out.data_ptr(), ws.data_ptr(), ws.numel(),
                                   _stream_handle(ifs.device)), "im_build_tsum")
    return out


def im_build_repaired(ifs, dm_mask, A, wfs: Wfs, threshold: float = 0.999999, out=None, ws=None):
    """IM of a pre-masked IF stack with the edge repair of Sec. 2.3 (see
    ``synim_im_build_repaired``); ``dm_mask`` is the DM-side 0/1 mask [H_in][W_in]."""
    torch = _torch()
    lib = load()
    _dev_f32(ifs, "ifs")
    n, H_in, W_in = ifs.shape
    if tuple(dm_mask.shape) != (H_in, W_in) or dm_mask.dtype != torch.uint8 or not dm_mask.is_cuda:
        raise ValueError("dm_mask must be a uint8 GPU tensor of the IF grid's shape")
    if out is None:
        out = torch.empty((n, 2 * wfs.n_valid), dtype=torch.float32, device=ifs.device)
    s = wfs.struct()
    a = _affine_struct(A)
    if ws is None:
        nb = C.c_size_t(0)
        _check(lib.synim_im_repaired_workspace(C.byref(s), C.byref(a), C.byref(nb)),
               "im_repaired_workspace")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=ifs.device)
    _check(lib.synim_im_build_repaired(ifs.data_ptr(), n, H_in, W_in, dm_mask.data_ptr(),
                                       float(threshold), C.byref(a), C.byref(s), out.data_ptr(),
                                       ws.data_ptr(), ws.numel(), _stream_handle(ifs.device)),
           "im_build_repaired")
    return out


def _dA_structs(dA):
    arr = (_abi.SynimAffine * 4)()
    for j in range(4):
        arr[j] = _affine_struct(dA[j])
    return arr


def im_jacobian(ifs, A, dA, wfs: Wfs, with_im: bool = True, ws=None):
    """(IM or None, dIM [4][n_act][2N]) for the derivative maps dA [4x2x3]."""
    torch = _torch()
    lib = load()
    _dev_f32(ifs, "ifs")
    n, H_in, W_in = ifs.shape
    nv2 = 2 * wfs.n_valid
    im = torch.empty((n, nv2), dtype=torch.float32, device=ifs.device) if with_im else None
    dim = torch.empty((4, n, nv2), dtype=torch.float32, device=ifs.device)
    ws = _workspace(wfs, A, 5, ws, ifs.device)
    s = wfs.struct()
    a = _affine_struct(A)
    _check(lib.synim_im_jacobian(ifs.data_ptr(), n, H_in, W_in, C.byref(a), _dA_structs(dA),
                                 C.byref(s), im.data_ptr() if im is not None else None,
                                 dim.data_ptr(), ws.data_ptr(), ws.numel(),
                                 _stream_handle(ifs.device)), "im_jacobian")
    return im, dim


def im_vjp(ifs, A, dA, wfs: Wfs, grad_im, ws=None):
    """grad_theta [4] (float64, device) = <grad_im, dIM/dtheta_j>."""
    torch = _torch()
    lib = load()
    _dev_f32(ifs, "ifs")
    _dev_f32(grad_im, "grad_im")
    n, H_in, W_in = ifs.shape
    out = torch.empty(4, dtype=torch.float64, device=ifs.device)
    ws = _workspace(wfs, A, 5, ws, ifs.device)
    s = wfs.struct()
    a = _affine_struct(A)
    _check(lib.synim_im_vjp(ifs.data_ptr(), n, H_in, W_in, C.byref(a), _dA_structs(dA),
                            C.byref(s), grad_im.data_ptr(), out.data_ptr(), ws.data_ptr(),
                            ws.numel(), _stream_handle(ifs.device)), "im_vjp")
    return out


def im_plan(wfs: Wfs, A, dA=None, planes: int = 1, ws=None, device="cuda", grid=(0, 0)):
    """Build the folded-geometry plan in a (new or given) workspace tensor.

    ``grid`` = (H_in, W_in) of the IF stacks the plan will stream, for the
    out-of-grid sample count of :func:`plan_oob`; (0, 0) leaves it uncounted."""
    lib = load()
    ws = _workspace(wfs, A, planes, ws, device)
    s = wfs.struct()
    a = _affine_struct(A)
    d = _dA_structs(dA) if dA is not None else None
    _check(lib.synim_im_plan(C.byref(s), C.byref(a), d, planes, int(grid[0]), int(grid[1]),
                             ws.data_ptr(), ws.numel(), _stream_handle(ws.device)), "im_plan")
    return ws


def im_apply(ifs, A, wfs: Wfs, ws, planes: int = 1, plane: int = 0, out=None):
    """Stream ifs through one plane of a plan built by :func:`im_plan`."""
    torch = _torch()
    lib = load()
    _dev_f32(ifs, "ifs")
    n, H_in, W_in = ifs.shape
    if out is None:
        out = torch.empty((n, 2 * wfs.n_valid), dtype=torch.float32, device=ifs.device)
    s = wfs.struct()
    a = _affine_struct(A)
    _check(lib.synim_im_apply(ifs.data_ptr(), n, H_in, W_in, C.byref(a), C.byref(s), planes,
                              plane, out.data_ptr(), ws.data_ptr(), ws.numel(),
                              _stream_handle(ifs.device)), "im_apply")
    return out


def im_autotune(ifs, A, wfs: Wfs, max_candidates: int = 8, ws=None):
    """Time candidate kernel configurations on ``ifs`` and cache the fastest.

    Returns the list of per-candidate times (ms) in the order tried."""
    torch = _torch()
    lib = load()
    _dev_f32(ifs, "ifs")
    n, H_in, W_in = ifs.shape
    out = torch.empty((n, 2 * wfs.n_valid), dtype=torch.float32, device=ifs.device)
    ws = _workspace(wfs, A, 1, ws, ifs.device)
    times = (C.c_float * max_candidates)()
    tried = C.c_int(0)
    s = wfs.struct()
    a = _affine_struct(A)
    _check(lib.synim_im_autotune(ifs.data_ptr(), n, H_in, W_in, C.byref(a), C.byref(s),
                                 out.data_ptr(), ws.data_ptr(), ws.numel(), max_candidates, times,
                                 C.byref(tried), _stream_handle(ifs.device)), "im_autotune")
    return [float(times[i]) for i in range(tried.value)]


_CFG_KEYS = ("block", "lanes_per_subap", "patch_rows", "patch_cols", "tile_x", "tile_y", "stages",
             "schedule", "dma_per_wave", "pack")
_NCFG = len(_CFG_KEYS)


def im_config(wfs: Wfs, A) -> dict:
    """Kernel configuration plan/apply would use for this geometry now."""
    lib = load()
    o = (C.c_int * _NCFG)()
    s = wfs.struct()
    a = _affine_struct(A)
    _check(lib.synim_im_config(C.byref(s), C.byref(a), o), "im_config")
    return dict(zip(_CFG_KEYS, o[:_NCFG]))


def im_candidates(wfs: Wfs, A, max_out: int = 256) -> list:
    """Candidate kernel configurations in the autotuner's order."""
    lib = load()
    o = (C.c_int * (_NCFG * max_out))()
    n = C.c_int(0)
    s = wfs.struct()
    a = _affine_struct(A)
    _check(lib.synim_im_candidates(C.byref(s), C.byref(a), o, max_out, C.byref(n)),
           "im_candidates")
    return [dict(zip(_CFG_KEYS, o[_NCFG * i:_NCFG * (i + 1)])) for i in range(n.value)]


def im_set_config(wfs: Wfs, A, config: dict):
    """Pin one of :func:`im_candidates` for this geometry."""
    lib = load()
    o = (C.c_int * _NCFG)(*[int(config[k]) for k in _CFG_KEYS])
    s = wfs.struct()
    a = _affine_struct(A)
    _check(lib.synim_im_set_config(C.byref(s), C.byref(a), o), "im_set_config")


def autotune_clear():
    load().synim_autotune_clear()


def autotune_export() -> list:
    """The autotune cache as a list of ints (see ``synim_autotune_export``)."""
    lib = load()
    n = C.c_int(0)
    _check(lib.synim_autotune_export(None, 0, C.byref(n)), "autotune_export")
    buf = (C.c_int32 * max(1, n.value))()
    _check(lib.synim_autotune_export(buf, n.value, C.byref(n)), "autotune_export")
    return [int(buf[i]) for i in range(n.value)]


def autotune_import(record) -> None:
    """Merge a record from :func:`autotune_export` into the cache."""
    rec = [int(x) for x in record]
    buf = (C.c_int32 * max(1, len(rec)))(*rec)
    _check(load().synim_autotune_import(buf, len(rec)), "autotune_import")


def autotune_save(path: str, device_name: str = "") -> None:
    """Write the autotune cache to a JSON file (with the device it was measured
    on, as given)."""
    import json
    with open(path, "w") as f:
        json.dump({"format": 1, "device": device_name, "record": autotune_export()}, f)


def autotune_load(path: str, device_name: str = "") -> bool:
    """Merge a cache written by :func:`autotune_save`; False (nothing merged)
    when it was measured on another device than ``device_name`` (when both
    are given)."""
    import json
    with open(path) as f:
        d = json.load(f)
    if d.get("format") != 1:
        raise ValueError("not an autotune cache file")
    if device_name and d.get("device") and d["device"] != device_name:
        return False
    autotune_import(d["record"])
    return True


def plan_status(ws) -> int:
    """Device status word of the last plan built in ``ws`` (synchronises)."""
    lib = load()
    v = C.c_int(0)
    _check(lib.synim_plan_status(ws.data_ptr(), C.byref(v), _stream_handle(ws.device)),
           "plan_status")
    return int(v.value)


def plan_oob(ws) -> int:
    """Out-of-grid samples of the last plan built in ``ws`` (synchronises).

    The C call returns SYNIM_E_OOB when the count is non-zero (its strict
    check); here the count itself is returned."""
    lib = load()
    v = C.c_int64(0)
    rc = lib.synim_plan_oob(ws.data_ptr(), C.byref(v), _stream_handle(ws.device))
    if rc != STATUS_OOB:
        _check(rc, "plan_oob")
    return int(v.value)


# ------------------------------------------------------ tomographic projection
def _proj_components(comps):
    """comps: list of (basis GPU float32 [n][H][W], altitude m, pixel m)."""
    arr = (_abi.SynimProjComponent * len(comps))()
    for i, (F, h, s) in enumerate(comps):
        _dev_f32(F, "basis")
        n, H, W = F.shape
        arr[i] = _abi.SynimProjComponent(F.data_ptr(), n, H, W, float(h), float(s))
    return arr


def _host_u8(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint8))
    return a, a.ctypes.data_as(C.c_void_p)


def proj_matrix(comps, dirs, pupil, pupil_pixel_m: float, bin: int = 1):
    """Transposed projection matrix Pt [sum n][rows] (GPU float64) of the components
    over the pupil (host 0/1 array) along every direction (radians, [n_dir][2])."""
    torch = _torch()
    lib = load()
    arr = _proj_components(comps)
    pu, pp = _host_u8(pupil)
    Hp, Wp = pu.shape
    d = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 2))
    rows = C.c_int(0)
    _check(lib.synim_proj_rows(pp, Hp, Wp, bin, d.shape[0], C.byref(rows)), "proj_rows")
    nb = C.c_size_t(0)
    _check(lib.synim_proj_workspace(arr, len(comps), None, 0, d.shape[0], pp, Hp, Wp, bin,
                                    C.byref(nb)), "proj_workspace")
    dev = comps[0][0].device
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    ncol = sum(int(F.shape[0]) for F, _, _ in comps)
    Pt = torch.empty((ncol, rows.value), dtype=torch.float64, device=dev)
    _check(lib.synim_proj_matrix(arr, len(comps), d.ctypes.data_as(C.c_void_p), d.shape[0], pp,
                                 Hp, Wp, float(pupil_pixel_m), bin, Pt.data_ptr(), rows.value,
                                 ws.data_ptr(), ws.numel(), _stream_handle(dev)), "proj_matrix")
    return Pt


def proj_opt(dms, layers, dirs, pupil, pupil_pixel_m: float, lam: float, bin: int = 1,
             ws=None):
    """P_opt [sum n_dm][sum n_layer] (GPU float64) of Sec. 2.5."""
    torch = _torch()
    lib = load()
    a_dm, a_l = _proj_components(dms), _proj_components(layers)
    pu, pp = _host_u8(pupil)
    Hp, Wp = pu.shape
    d = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 2))
    dev = dms[0][0].device
    if ws is None:
        nb = C.c_size_t(0)
        _check(lib.synim_proj_workspace(a_dm, len(dms), a_l, len(layers), d.shape[0], pp, Hp, Wp,
                                        bin, C.byref(nb)), "proj_workspace")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    ndm = sum(int(F.shape[0]) for F, _, _ in dms)
    nl = sum(int(F.shape[0]) for F, _, _ in layers)
    out = torch.empty((ndm, nl), dtype=torch.float64, device=dev)
    _check(lib.synim_proj_opt(a_dm, len(dms), a_l, len(layers), d.ctypes.data_as(C.c_void_p),
                              d.shape[0], pp, Hp, Wp, float(pupil_pixel_m), bin, float(lam),
                              out.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(dev)),
           "proj_opt")
    return out


def proj_workspace_bytes(dms, layers, n_dir: int, pupil, bin: int = 1) -> int:
    lib = load()
    a_dm, a_l = _proj_components(dms), _proj_components(layers)
    pu, pp = _host_u8(pupil)
    nb = C.c_size_t(0)
    _check(lib.synim_proj_workspace(a_dm, len(dms), a_l, len(layers), n_dir, pp, pu.shape[0],
                                    pu.shape[1], bin, C.byref(nb)), "proj_workspace")
    return int(nb.value)


def gemm_f64(M, N, K, alpha, X, sxk, sxm, Y, syk, syn, beta, Cm, ldc):
    """C[m][n] = alpha sum_k X(k,m) Y(k,n) + beta C[m][n] on GPU float64 tensors (strides
    in elements)."""
    lib = load()
    _check(lib.synim_gemm_f64(M, N, K, float(alpha), X.data_ptr(), sxk, sxm, Y.data_ptr(), syk,
                              syn, float(beta), Cm.data_ptr(), ldc, _stream_handle(Cm.device)),
           "gemm_f64")
    return Cm


def potrf_f64(A, status):
    """In-place lower Cholesky of the GPU float64 square matrix A; status int32 GPU [1]."""
    lib = load()
    n = A.shape[0]
    _check(lib.synim_potrf_f64(A.data_ptr(), n, A.stride(0), status.data_ptr(),
                               _stream_handle(A.device)), "potrf_f64")
    return A


def potrs_f64(L, B):
    """B <- (L L^T)^-1 B in place (GPU float64, row-major)."""
    lib = load()
    _check(lib.synim_potrs_f64(L.data_ptr(), L.shape[0], L.stride(0), B.data_ptr(), B.shape[1],
                               B.stride(0), _stream_handle(B.device)), "potrs_f64")
    return B


# --------------------------------------------------------------- multi-pair
class Batch:
    """Every (WFS, DM) pair of a multi-WFS system built in one persistent launch.

    ``wfs``: list of :class:`Wfs`; ``stacks``: list of IF stacks (GPU float32
    [n_act][H][W]); ``pairs``: list of (wfs index, dm index, map [2x3]).
    ``outs[i]`` is pair i's IM [n_act(dm)][2 N(wfs)] (allocated if not given).
    The maps stay in device memory: :meth:`set_maps` followed by
    :meth:`run_graph` replays the captured graph without re-capture.
    """

    def __init__(self, wfs, stacks, pairs, outs=None, device="cuda"):
        torch = _torch()
        lib = load()
        self._wfs = list(wfs)
        self._stacks = [_dev_f32(t, "stack") for t in stacks]
        self.n_pairs = len(pairs)
        if outs is None:
            outs = [torch.empty((self._stacks[d].shape[0], 2 * self._wfs[w].n_valid),
                                dtype=torch.float32, device=device) for (w, d, _) in pairs]
        self.outs = list(outs)
        self._w = (_abi.SynimWfs * len(self._wfs))(*[w.struct() for w in self._wfs])
        self._d = (_abi.SynimDm * len(self._stacks))(
            *[_abi.SynimDm(t.data_ptr(), t.shape[0], t.shape[1], t.shape[2]) for t in self._stacks])
        self._p = (_abi.SynimPair * self.n_pairs)(
            *[_abi.SynimPair(w, d, _affine_struct(A), o.data_ptr())
              for (w, d, A), o in zip(pairs, self.outs)])
        n = C.c_size_t(0)
        _check(lib.synim_batch_workspace(self._w, len(self._wfs), self._d, len(self._stacks),
                                         self._p, self.n_pairs, C.byref(n)), "batch_workspace")
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=device)
        self._h = C.c_void_p(0)
        self._stream = torch.cuda.current_stream(self.ws.device)
        _check(lib.synim_batch_create(self._w, len(self._wfs), self._d, len(self._stacks),
                                      self._p, self.n_pairs, self.ws.data_ptr(), self.ws.numel(),
                                      self._stream.cuda_stream, C.byref(self._h)), "batch_create")

    def _sh(self):
        return _torch().cuda.current_stream(self.ws.device).cuda_stream

    def set_maps(self, maps):
        arr = (_abi.SynimAffine * self.n_pairs)(*[_affine_struct(A) for A in maps])
        _check(load().synim_batch_set_maps(self._h, arr, self._sh()), "batch_set_maps")

    def run(self):
        _check(load().synim_batch_run(self._h, self._sh()), "batch_run")
        return self.outs

    def run_graph(self):
        """Replay the captured graph (captured on the first call).

        Graph capture needs a stream other than the null stream, so the graph
        runs on a side stream of the batch, ordered after the caller's current
        stream and before its later work."""
        torch = _torch()
        cur = torch.cuda.current_stream(self.ws.device)
        if not hasattr(self, "_side"):
            self._side = torch.cuda.Stream(device=self.ws.device)
        self._side.wait_stream(cur)
        _check(load().synim_batch_run_graph(self._h, self._side.cuda_stream), "batch_run_graph")
        cur.wait_stream(self._side)
        return self.outs

    def status(self) -> int:
        v = C.c_int(0)
        _check(load().synim_batch_status(self._h, C.byref(v), self._sh()), "batch_status")
        return int(v.value)

    def oob(self) -> int:
        """Out-of-grid samples of the last run, summed over the pairs (synchronises)."""
        v = C.c_int64(0)
        rc = load().synim_batch_oob(self._h, C.byref(v), self._sh())
        if rc != STATUS_OOB:
            _check(rc, "batch_oob")
        return int(v.value)

    def autotune(self, max_variants: int = 6):
        t = (C.c_float * max_variants)()
        n = C.c_int(0)
        _check(load().synim_batch_autotune(self._h, max_variants, t, C.byref(n), self._sh()),
               "batch_autotune")
        return [float(t[i]) for i in range(n.value)]

    def config(self) -> dict:
        o = (C.c_int * 6)()
        _check(load().synim_batch_config(self._h, o), "batch_config")
        return dict(block=o[0], lanes_per_subap=o[1], stages=o[2], grid=o[3],
                    dma_per_wave=o[4], pack=o[5])

    def parts(self) -> int:
        """Launches per run: 1, or the patch-size parts of a split batch."""
        n = C.c_int(0)
        _check(load().synim_batch_parts(self._h, C.byref(n)), "batch_parts")
        return int(n.value)

    def close(self):
        if self._h and self._h.value:
            load().synim_batch_destroy(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ MLP
class Mlp:
    """Packed-parameter MLP n_in -> h1 -> h2 -> n_out (HIP forward/backward/Adam).

    ``segments`` = ((seg0, len0), (seg1, len1)): compact input column c feeds
    input seg0 + c (c < len0) or seg1 + c - len0; all other inputs are zero."""

    def __init__(self, n_in, h1, h2, n_out, segments):
        (s0, l0), (s1, l1) = segments
        self.desc = _abi.SynimMlp(n_in, h1, h2, n_out, s0, l0, s1, l1)
        self.n_params = int(load().synim_mlp_param_count(C.byref(self.desc)))
        if self.n_params == 0:
            raise ValueError("invalid MLP description")

    @property
    def n_compact(self) -> int:
        return self.desc.len0 + self.desc.len1

    def layout(self):
        d = self.desc
        sizes = [d.h1 * d.n_in, d.h1, d.h2 * d.h1, d.h2, d.n_out * d.h2, d.n_out]
        offs = np.cumsum([0] + sizes)
        return [(int(offs[i]), int(offs[i + 1])) for i in range(6)]

    def scratch(self, B, device="cuda"):
        torch = _torch()
        n = int(load().synim_mlp_scratch_floats(C.byref(self.desc), B))
        return torch.empty(n, dtype=torch.float32, device=device)

    def forward(self, params, x, scratch, out=None):
        torch = _torch()
        _dev_f32(params, "params")
        _dev_f32(x, "x")
        B = x.shape[0]
        if out is None:
            out = torch.empty((B, self.desc.n_out), dtype=torch.float32, device=x.device)
        _check(load().synim_mlp_forward(C.byref(self.desc), params.data_ptr(), x.data_ptr(), B,
                                        scratch.data_ptr(), out.data_ptr(),
                                        _stream_handle(x.device)), "mlp_forward")
        return out

    def backward(self, params, x, scratch, y, t, grads, loss=None):
        _check(load().synim_mlp_backward(C.byref(self.desc), params.data_ptr(), x.data_ptr(),
                                         x.shape[0], scratch.data_ptr(), y.data_ptr(),
                                         t.data_ptr(), grads.data_ptr(),
                                         loss.data_ptr() if loss is not None else None,
                                         _stream_handle(x.device)), "mlp_backward")
        return grads


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(load().synim_adam_step(params.data_ptr(), grads.data_ptr(), m.data_ptr(),
                                  v.data_ptr(), params.numel(), int(step), float(lr),
                                  float(beta1), float(beta2), float(eps),
                                  _stream_handle(params.device)), "adam_step")


# ------------------------------------------------------- misregistration
MISREG_GN, MISREG_MLP, MISREG_MLP_GN = 0, 1, 2


class Misreg:
    """Batched misregistration estimation from probe slopes (GN, MLP, MLP+GN).

    ``probes``: GPU float32 [n_probe][H][W] probe phase maps; ``wfs``:
    :class:`Wfs`; ``lo``/``hi``: label box (shift x px, shift y px, rot rad,
    mag).  ``mlp`` = (Mlp, params, feat_mean, feat_std, feat_len) or None."""

    def __init__(self, wfs: Wfs, probes, lo, hi, max_batch=1, max_iter=20, tol=1e-6,
                 kappa=1.0, mlp=None, gn_batched=False):
        torch = _torch()
        lib = load()
        self.wfs = wfs
        self.probes = _dev_f32(probes, "probes")
        self.mlp = mlp
        d = _abi.SynimMisregDesc()
        d.wfs = wfs.struct()
        d.probes = probes.data_ptr()
        d.n_probe, d.H_in, d.W_in = probes.shape
        d.kappa = float(kappa)
        d.max_batch = int(max_batch)
        for j in range(4):
            d.theta_lo[j] = float(lo[j])
            d.theta_hi[j] = float(hi[j])
        d.max_iter = int(max_iter)
        d.tol = float(tol)
        d.gn_batched = 1 if gn_batched else 0
        if mlp is not None:
            net, params, mean, std, feat_len = mlp
            d.mlp_params = params.data_ptr()
            d.h1, d.h2 = net.desc.h1, net.desc.h2
            d.feat_len = int(feat_len)
            d.feat_mean = mean.data_ptr()
            d.feat_std = std.data_ptr()
        self.desc = d
        self.M = d.n_probe * 2 * wfs.n_valid
        n = C.c_size_t(0)
        _check(lib.synim_misreg_workspace(C.byref(d), C.byref(n)), "misreg_workspace")
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=probes.device)
        self._h = C.c_void_p(0)
        _check(lib.synim_misreg_create(C.byref(d), self.ws.data_ptr(), self.ws.numel(),
                                       _stream_handle(probes.device), C.byref(self._h)),
               "misreg_create")
        self._side = torch.cuda.Stream(device=probes.device)

    def slopes(self, theta, jac=False):
        """S [B][M] (and J [B][4][M]) at theta (GPU float64 [B][4])."""
        torch = _torch()
        B = theta.shape[0]
        s = torch.empty((B, self.M), dtype=torch.float32, device=theta.device)
        j = torch.empty((B, 4, self.M), dtype=torch.float32, device=theta.device) if jac else None
        _check(load().synim_misreg_slopes(self._h, theta.contiguous().data_ptr(), B,
                                          s.data_ptr(), j.data_ptr() if jac else None,
                                          _stream_handle(theta.device)), "misreg_slopes")
        return (s, j) if jac else s

    def features(self, slopes, mean=None, std=None):
        torch = _torch()
        B = slopes.shape[0]
        x = torch.empty((B, self.M), dtype=torch.float32, device=slopes.device)
        _check(load().synim_misreg_features(
            self._h, slopes.data_ptr(), B, mean.data_ptr() if mean is not None else None,
            std.data_ptr() if std is not None else None, x.data_ptr(),
            _stream_handle(slopes.device)), "misreg_features")
        return x

    def infer(self, slopes, mode=MISREG_GN, iter_cap=0, use_graph=True, out=None):
        """(theta [B][4] float64, iterations [B] int32) on the GPU.

        ``out`` = (theta, iterations) tensors to write; reusing them lets the
        graph captured for these arrays replay with no copies."""
        torch = _torch()
        _dev_f32(slopes, "slopes")
        B = slopes.shape[0]
        if out is not None:
            th, it = out
        else:
            th = torch.empty((B, 4), dtype=torch.float64, device=slopes.device)
            it = torch.empty(B, dtype=torch.int32, device=slopes.device)
        if use_graph:
            cur = torch.cuda.current_stream(slopes.device)
            self._side.wait_stream(cur)
            sh = self._side.cuda_stream
        else:
            sh = _stream_handle(slopes.device)
        _check(load().synim_misreg_infer(self._h, slopes.data_ptr(), B, mode, th.data_ptr(),
                                         it.data_ptr(), int(iter_cap), 1 if use_graph else 0, sh),
               "misreg_infer")
        if use_graph:
            cur.wait_stream(self._side)
        return th, it

    def status(self) -> int:
        v = C.c_int(0)
        _check(load().synim_misreg_status(self._h, C.byref(v), _stream_handle(self.ws.device)),
               "misreg_status")
        return int(v.value)

    def unconverged(self) -> int:
        """Samples of the last :meth:`infer` whose Gauss-Newton loop stopped without
        converging (synchronises; the C call signals them with SYNIM_E_NOT_CONVERGED)."""
        v = C.c_int32(0)
        rc = load().synim_misreg_unconverged(self._h, C.byref(v), _stream_handle(self.ws.device))
        if rc != STATUS_NOT_CONVERGED:
            _check(rc, "misreg_unconverged")
        return int(v.value)

    def close(self):
        if self._h and self._h.value:
            load().synim_misreg_destroy(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
