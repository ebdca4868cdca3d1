"""ctypes declarations of the C ABI in ``include/synim.h`` (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

# the in-tree build; SYNIM_LIB names another build of the same sources
LIB_PATH = os.environ.get(
    "SYNIM_LIB", os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynim.so"))


class SynimAffine(C.Structure):
    _fields_ = [("A", (C.c_double * 2) * 2), ("b", C.c_double * 2)]


class SynimMisreg(C.Structure):
    _fields_ = [("shift_x", C.c_double), ("shift_y", C.c_double), ("rot", C.c_double),
                ("mag", C.c_double)]


class SynimGeometry(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "dm_shift_x", "dm_shift_y", "dm_rot", "dm_mag", "cone_scale", "footprint_x",
        "footprint_y", "wfs_shift_x", "wfs_shift_y", "wfs_rot", "wfs_mag_x", "wfs_mag_y",
        "kappa")]


class SynimWfs(C.Structure):
    _fields_ = [("n_sub_x", C.c_int32), ("n_sub_y", C.c_int32), ("p", C.c_int32),
                ("n_valid", C.c_int32), ("valid_idx", C.c_void_p), ("pupil", C.c_void_p)]


class SynimDm(C.Structure):
    _fields_ = [("ifs", C.c_void_p), ("n_act", C.c_int32), ("H_in", C.c_int32), ("W_in", C.c_int32)]


class SynimPair(C.Structure):
    _fields_ = [("wfs", C.c_int32), ("dm", C.c_int32), ("A", SynimAffine), ("im", C.c_void_p)]


class SynimProjComponent(C.Structure):
    _fields_ = [("basis", C.c_void_p), ("n", C.c_int32), ("H", C.c_int32), ("W", C.c_int32),
                ("altitude_m", C.c_double), ("pixel_m", C.c_double)]


class SynimMlp(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("n_in", "h1", "h2", "n_out", "seg0", "len0", "seg1",
                                         "len1")]


class SynimMisregDesc(C.Structure):
    _fields_ = [("wfs", SynimWfs), ("probes", C.c_void_p), ("n_probe", C.c_int32),
                ("H_in", C.c_int32), ("W_in", C.c_int32), ("kappa", C.c_double),
                ("max_batch", C.c_int32), ("theta_lo", C.c_double * 4),
                ("theta_hi", C.c_double * 4), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("mlp_params", C.c_void_p), ("h1", C.c_int32), ("h2", C.c_int32),
                ("feat_len", C.c_int32), ("feat_mean", C.c_void_p), ("feat_std", C.c_void_p),
                ("gn_batched", C.c_int32)]


P = C.c_void_p
I = C.c_int
SZ = C.c_size_t

# name -> (restype, argtypes); every function declared in include/synim.h
SIGNATURES = {
    "synim_status_str": (C.c_char_p, [I]),
    "synim_version": (I, []),
    "synim_affine_from_misreg": (I, [C.POINTER(SynimMisreg), I, I, I, I, C.c_double,
                                     C.POINTER(SynimAffine), C.POINTER(SynimAffine)]),
    "synim_affine_from_geometry": (I, [C.POINTER(SynimGeometry), I, I, I, I,
                                       C.POINTER(SynimAffine)]),
    "synim_affine_warp": (I, [P, I, I, I, C.POINTER(SynimAffine), I, I, I, P, P, P]),
    "synim_sa_slopes": (I, [P, I, C.POINTER(SynimWfs), P, P]),
    "synim_im_workspace": (I, [C.POINTER(SynimWfs), C.POINTER(SynimAffine), I, C.POINTER(SZ)]),
    "synim_im_build": (I, [P, I, I, I, C.POINTER(SynimAffine), C.POINTER(SynimWfs), P, P, SZ, P]),
    "synim_im_build_tsum": (I, [P, I, I, I, C.POINTER(SynimAffine), C.POINTER(SynimWfs), P, P,
                                SZ, P]),
    "synim_im_repaired_workspace": (I, [C.POINTER(SynimWfs), C.POINTER(SynimAffine),
                                        C.POINTER(SZ)]),
    "synim_im_build_repaired": (I, [P, I, I, I, P, C.c_double, C.POINTER(SynimAffine),
                                    C.POINTER(SynimWfs), P, P, SZ, P]),
    "synim_im_build_noalloc": (I, [P, I, I, I, C.POINTER(SynimAffine), C.POINTER(SynimWfs), P,
                                   P]),
    "synim_im_jacobian": (I, [P, I, I, I, C.POINTER(SynimAffine), C.POINTER(SynimAffine),
                              C.POINTER(SynimWfs), P, P, P, SZ, P]),
    "synim_im_vjp": (I, [P, I, I, I, C.POINTER(SynimAffine), C.POINTER(SynimAffine),
                         C.POINTER(SynimWfs), P, P, P, SZ, P]),
    "synim_im_plan": (I, [C.POINTER(SynimWfs), C.POINTER(SynimAffine), C.POINTER(SynimAffine),
                          I, I, I, P, SZ, P]),
    "synim_im_apply": (I, [P, I, I, I, C.POINTER(SynimAffine), C.POINTER(SynimWfs), I, I, P, P,
                           SZ, P]),
    "synim_plan_status": (I, [P, C.POINTER(I), P]),
    "synim_plan_oob": (I, [P, C.POINTER(C.c_int64), P]),
    "synim_im_autotune": (I, [P, I, I, I, C.POINTER(SynimAffine), C.POINTER(SynimWfs), P, P, SZ,
                              I, C.POINTER(C.c_float), C.POINTER(I), P]),
    "synim_im_config": (I, [C.POINTER(SynimWfs), C.POINTER(SynimAffine), C.POINTER(I)]),
    "synim_autotune_clear": (None, []),
    "synim_autotune_export": (I, [C.POINTER(C.c_int32), I, C.POINTER(I)]),
    "synim_autotune_import": (I, [C.POINTER(C.c_int32), I]),
    "synim_batch_workspace": (I, [C.POINTER(SynimWfs), I, C.POINTER(SynimDm), I,
                                  C.POINTER(SynimPair), I, C.POINTER(SZ)]),
    "synim_batch_create": (I, [C.POINTER(SynimWfs), I, C.POINTER(SynimDm), I,
                               C.POINTER(SynimPair), I, P, SZ, P, C.POINTER(P)]),
    "synim_batch_set_maps": (I, [P, C.POINTER(SynimAffine), P]),
    "synim_batch_run": (I, [P, P]),
    "synim_batch_run_graph": (I, [P, P]),
    "synim_batch_status": (I, [P, C.POINTER(I), P]),
    "synim_batch_oob": (I, [P, C.POINTER(C.c_int64), P]),
    "synim_batch_autotune": (I, [P, I, C.POINTER(C.c_float), C.POINTER(I), P]),
    "synim_batch_config": (I, [P, C.POINTER(I)]),
    "synim_batch_parts": (I, [P, C.POINTER(I)]),
    "synim_batch_destroy": (None, [P]),
    "synim_proj_rows": (I, [P, I, I, I, I, C.POINTER(I)]),
    "synim_proj_workspace": (I, [C.POINTER(SynimProjComponent), I, C.POINTER(SynimProjComponent),
                                 I, I, P, I, I, I, C.POINTER(SZ)]),
    "synim_proj_matrix": (I, [C.POINTER(SynimProjComponent), I, P, I, P, I, I, C.c_double, I, P,
                              C.c_long, P, SZ, P]),
    "synim_proj_opt": (I, [C.POINTER(SynimProjComponent), I, C.POINTER(SynimProjComponent), I, P,
                           I, P, I, I, C.c_double, I, C.c_double, P, P, SZ, P]),
    "synim_gemm_f64": (I, [I, I, I, C.c_double, P, C.c_long, C.c_long, P, C.c_long, C.c_long,
                           C.c_double, P, C.c_long, P]),
    "synim_potrf_f64": (I, [P, I, C.c_long, P, P]),
    "synim_potrs_f64": (I, [P, I, C.c_long, P, I, C.c_long, P]),
    "synim_mlp_param_count": (SZ, [C.POINTER(SynimMlp)]),
    "synim_mlp_scratch_floats": (SZ, [C.POINTER(SynimMlp), I]),
    "synim_mlp_forward": (I, [C.POINTER(SynimMlp), P, P, I, P, P, P]),
    "synim_mlp_backward": (I, [C.POINTER(SynimMlp), P, P, I, P, P, P, P, P, P]),
    "synim_adam_step": (I, [P, P, P, P, SZ, I, C.c_double, C.c_double, C.c_double, C.c_double,
                            P]),
    "synim_misreg_workspace": (I, [C.POINTER(SynimMisregDesc), C.POINTER(SZ)]),
    "synim_misreg_create": (I, [C.POINTER(SynimMisregDesc), P, SZ, P, C.POINTER(P)]),
    "synim_misreg_slopes": (I, [P, P, I, P, P, P]),
    "synim_misreg_features": (I, [P, P, I, P, P, P, P]),
    "synim_misreg_infer": (I, [P, P, I, I, P, P, I, I, P]),
    "synim_misreg_status": (I, [P, C.POINTER(I), P]),
    "synim_misreg_unconverged": (I, [P, C.POINTER(C.c_int32), P]),
    "synim_misreg_destroy": (None, [P]),
    "synim_im_candidates": (I, [C.POINTER(SynimWfs), C.POINTER(SynimAffine), C.POINTER(I), I,
                                C.POINTER(I)]),
    "synim_im_set_config": (I, [C.POINTER(SynimWfs), C.POINTER(SynimAffine), C.POINTER(I)]),
}


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library not found at {path}; build it with `python -m paper_2606_07759_amd.build`")
    # torch first: its HIP runtime is then the one libsynim.so binds to (same
    # soname).  Loaded the other way round, the process would hold two HIP
    # runtimes, and torch's streams and allocations would be foreign to the
    # library's (its host copies of torch device memory fail).
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib
