"""Seeded synthetic inputs for the interaction-matrix (IM) path.

This module only *synthesises inputs*: pupil masks, valid-subaperture lists,
Gaussian influence-function (IF) stacks, misregistration parameters drawn from a
seed, multi-WFS pair geometry and Zernike probe commands.  It holds none of the
method's arithmetic (no warp, no finite differences, no slope means), so both the
FP64 oracle's tests and the HIP path's tests/bench can draw from it.

Conventions (shared by every consumer):

* pixel (row y, column x) has its centre at integer coordinates (x, y);
* a grid of n pixels has its centre at (n-1)/2;
* subaperture (u, v) of size p covers columns u*p..u*p+p-1 and rows v*p..v*p+p-1
  and is numbered row-major, ``k = v*n_sub_x + u``;
* all random draws use ``numpy.random.Generator(PCG64(seed))``.

The workloads restate the paper's configurations as concrete synthetic inputs:
an 8x8 SCAO Shack-Hartmann sensor, an ELT-scale 80x80 sensor on a 480-pixel
pupil with 28% central obscuration, and a 6-LGS / 3-DM MCAO geometry with cone
effect and off-axis footprints (paper Sec. 4, Sec. 2.1).  The real MORFEO IF
cubes and M4 modes are not available, so Gaussian IFs with 15% inter-actuator
coupling stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "SIGMA_PER_PITCH", "rng_for", "pupil_mask", "valid_subapertures",
    "ActuatorGrid", "actuator_grid", "if_stack", "if_single",
    "Geometry", "misreg_geometry", "ScaoConfig", "scao_small", "scao_elt",
    "McaoPair", "McaoConfig", "mcao", "zernike_noll", "probe_commands",
    "ProbeConfig", "probe_config", "draw_misreg_labels",
    "FourierMode", "fourier_modes", "fourier_mode_values", "fourier_stack",
    "fourier_stack_torch",
]

# IF(pitch) = 0.15 * IF(0) for a Gaussian exp(-r^2 / 2 sigma^2).
SIGMA_PER_PITCH = 1.0 / math.sqrt(2.0 * math.log(1.0 / 0.15))


def rng_for(seed: int) -> np.random.Generator:
    """The one random generator used for every seeded draw."""
    return np.random.Generator(np.random.PCG64(int(seed)))


# --------------------------------------------------------------------------- pupils
def pupil_mask(n: int, diameter: float, obscuration: float = 0.0,
               center_offset: Tuple[float, float] = (0.0, 0.0)) -> np.ndarray:
    """Binary annular pupil on an n x n grid (uint8).

    A pixel belongs to the pupil when its centre lies at radius r with
    ``obscuration*D/2 <= r <= D/2`` from the grid centre shifted by
    ``center_offset`` (x, y) pixels.
    """
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    r = np.hypot(x - c - center_offset[0], y - c - center_offset[1])
    inside = (r <= diameter / 2.0) & (r >= obscuration * diameter / 2.0)
    return inside.astype(np.uint8)


def valid_subapertures(pupil: np.ndarray, p: int, tau: float = 0.5) -> np.ndarray:
    """Row-major ids of subapertures whose illuminated fraction is >= tau (int32)."""
    h, w = pupil.shape
    if h % p or w % p:
        raise ValueError("pupil grid must be an exact multiple of the subaperture size")
    frac = pupil.reshape(h // p, p, w // p, p).astype(np.int64).sum(axis=(1, 3)) / float(p * p)
    return np.flatnonzero(frac.ravel() >= tau).astype(np.int32)


# ----------------------------------------------------------------------- IF stacks
@dataclass
class ActuatorGrid:
    grid_n: int                 # IF grid is grid_n x grid_n
    pitch: float                # actuator pitch, IF pixels
    x: np.ndarray               # actuator centres (float64, IF pixels)
    y: np.ndarray
    amp: np.ndarray             # per-actuator amplitude (float64)
    sigma: float                # Gaussian width, IF pixels

    @property
    def n_act(self) -> int:
        return int(self.x.size)


def actuator_grid(n_1d: int, pitch: float, grid_n: int, keep_radius: Optional[float] = None,
                  amp_jitter: float = 0.0, rng: Optional[np.random.Generator] = None) -> ActuatorGrid:
    """Square (Fried) actuator grid centred on the IF grid centre.

    Actuators further than ``keep_radius`` from the centre are dropped.
    Amplitudes are 1, or N(1, amp_jitter) drawn from ``rng`` in actuator order.
    """
    c = (grid_n - 1) / 2.0
    pos = c + pitch * (np.arange(n_1d, dtype=np.float64) - (n_1d - 1) / 2.0)
    X, Y = np.meshgrid(pos, pos)
    X, Y = X.ravel(), Y.ravel()
    if keep_radius is not None:
        keep = np.hypot(X - c, Y - c) <= keep_radius
        X, Y = X[keep], Y[keep]
    if amp_jitter > 0.0:
        if rng is None:
            raise ValueError("amplitude jitter needs a generator")
        amp = rng.normal(1.0, amp_jitter, size=X.size)
    else:
        amp = np.ones(X.size)
    return ActuatorGrid(grid_n, float(pitch), X, Y, amp, float(SIGMA_PER_PITCH * pitch))


def _profiles(grid: ActuatorGrid, sel: np.ndarray):
    """1-D Gaussian factors (float64) for the selected actuators."""
    t = np.arange(grid.grid_n, dtype=np.float64)
    s2 = 2.0 * grid.sigma * grid.sigma
    gx = np.exp(-((t[None, :] - grid.x[sel, None]) ** 2) / s2)
    gy = np.exp(-((t[None, :] - grid.y[sel, None]) ** 2) / s2)
    return gx, gy


def if_stack(grid: ActuatorGrid, a0: int = 0, a1: Optional[int] = None) -> np.ndarray:
    """float32 IF stack [a1-a0][grid_n][grid_n]: amp * gy (x) gx, rounded once to FP32.

    The product is formed in float64 in the order ``amp * (gy[:,None] * gx[None,:])``
    so that a device-side generator using the same 1-D factors is bit-identical.
    """
    a1 = grid.n_act if a1 is None else a1
    sel = np.arange(a0, a1)
    gx, gy = _profiles(grid, sel)
    out = grid.amp[sel, None, None] * (gy[:, :, None] * gx[:, None, :])
    return out.astype(np.float32)


def if_single(grid: ActuatorGrid, a: int) -> np.ndarray:
    return if_stack(grid, a, a + 1)[0]


def if_stack_torch(grid: ActuatorGrid, device, chunk: int = 256):
    """Same values as :func:`if_stack` built on a torch device, chunked.

    The 1-D factors are computed once on the host (float64) and the outer
    products are formed on the device in float64, then rounded to float32, so
    the result is bit-identical to the host generator.
    """
    import torch
    gx, gy = _profiles(grid, np.arange(grid.n_act))
    gx_t = torch.from_numpy(gx).to(device)
    gy_t = torch.from_numpy(gy).to(device)
    amp_t = torch.from_numpy(grid.amp).to(device)
    out = torch.empty((grid.n_act, grid.grid_n, grid.grid_n), dtype=torch.float32, device=device)
    for a0 in range(0, grid.n_act, chunk):
        a1 = min(grid.n_act, a0 + chunk)
        blk = amp_t[a0:a1, None, None] * (gy_t[a0:a1, :, None] * gx_t[a0:a1, None, :])
        out[a0:a1] = blk.to(torch.float32)
        del blk
    return out


# ------------------------------------------------------------------------ geometry
@dataclass
class Geometry:
    """Forward DM-grid -> WFS-grid chain, every part about its grid centre.

    1. DM placement:   v = dm_mag * R(dm_rot) u + dm_shift     (u: DM px from the DM centre)
    2. LGS footprint:  w = (v - footprint) / (kappa * cone_scale)
    3. WFS:            p_o - c_o = diag(wfs_mag_x, wfs_mag_y) R(wfs_rot) w + wfs_shift

    ``kappa`` is DM pixels per WFS pixel.  R(phi) rotates counter-clockwise in the
    (x=column, y=row) frame.  Plain SCAO misregistration (shift t in WFS px,
    rotation rho, magnification m) is dm_mag=m, dm_rot=rho, dm_shift=kappa*t.
    """
    dm_shift_x: float = 0.0
    dm_shift_y: float = 0.0
    dm_rot: float = 0.0
    dm_mag: float = 1.0
    cone_scale: float = 1.0
    footprint_x: float = 0.0
    footprint_y: float = 0.0
    wfs_shift_x: float = 0.0
    wfs_shift_y: float = 0.0
    wfs_rot: float = 0.0
    wfs_mag_x: float = 1.0
    wfs_mag_y: float = 1.0
    kappa: float = 1.0


def misreg_geometry(theta: Sequence[float], kappa: float = 1.0) -> Geometry:
    tx, ty, rho, m = (float(v) for v in theta)
    return Geometry(dm_shift_x=kappa * tx, dm_shift_y=kappa * ty, dm_rot=rho, dm_mag=m, kappa=kappa)


# ------------------------------------------------------------------- SCAO workloads
@dataclass
class ScaoConfig:
    name: str
    n_sub: int
    p: int
    pupil: np.ndarray           # uint8 [n_sub*p][n_sub*p]
    valid: np.ndarray           # int32 row-major subaperture ids
    grid: ActuatorGrid
    theta: Tuple[float, float, float, float]   # (shift x px, shift y px, rot rad, mag)
    kappa: float = 1.0

    @property
    def n_out(self) -> int:
        return self.n_sub * self.p

    @property
    def n_valid(self) -> int:
        return int(self.valid.size)


def scao_small() -> ScaoConfig:
    """8x8 subapertures of 10 px, 80-px circular pupil, 9x9 Fried DM on a 96^2 grid.

    Misregistration: shift (0.3, -0.2) px, rotation 0.5 deg, magnification 1.01.
    """
    pupil = pupil_mask(80, 80.0)
    valid = valid_subapertures(pupil, 10)
    grid = actuator_grid(9, 10.0, 96)
    theta = (0.3, -0.2, math.radians(0.5), 1.01)
    return ScaoConfig("scao_8x8", 8, 10, pupil, valid, grid, theta)


def scao_elt(seed: int = 0) -> ScaoConfig:
    """ELT-scale SCAO: 80x80 subapertures of 6 px on a 480-px pupil, 28% obscuration.

    DM: 81x81 grid at 6-px pitch on a 512^2 IF grid, actuators within one pitch of
    the pupil edge kept (5257), amplitudes N(1, 0.02).  Misregistration drawn from
    the seed: shift U(-1,1) px per axis, rotation U(-1,1) deg, magnification U(0.98,1.02).
    The draws happen in that order, then the amplitudes.
    """
    rng = rng_for(seed)
    theta = (float(rng.uniform(-1.0, 1.0)), float(rng.uniform(-1.0, 1.0)),
             math.radians(float(rng.uniform(-1.0, 1.0))), float(rng.uniform(0.98, 1.02)))
    pupil = pupil_mask(480, 480.0, 0.28)
    valid = valid_subapertures(pupil, 6)
    grid = actuator_grid(81, 6.0, 512, keep_radius=240.0 + 6.0, amp_jitter=0.02, rng=rng)
    return ScaoConfig(f"scao_elt_s{seed}", 80, 6, pupil, valid, grid, theta)


# ------------------------------------------------------------------- MCAO workload
@dataclass
class McaoPair:
    wfs: int
    dm: int
    geometry: Geometry


@dataclass
class McaoConfig:
    n_sub: int
    p: int
    pupils: List[np.ndarray]
    valids: List[np.ndarray]
    grids: List[ActuatorGrid]
    altitudes_m: List[float]
    pairs: List[McaoPair]
    pixel_scale_m: float
    lgs_height_m: float
    ring_radius_rad: float
    azimuths_rad: List[float]


def mcao(seed: int = 0, n_wfs: int = 6, n_sub: int = 68, p: int = 7) -> McaoConfig:
    """6 LGS WFS x 3 DMs (0 / 4 / 12.7 km) on a 39-m telescope.

    * WFS: n_sub x n_sub subapertures of p px (476-px pupil, 28% obscuration).
      LGS at 90 km on a 45-arcsec-radius ring at azimuths 0, 60, ..., 300 deg.
      Each WFS is clocked so that the radial (elongation) direction runs along a
      subaperture diagonal, and its pupil image is shifted by a seeded
      sub-subaperture offset U(-p/2, p/2) per axis, which makes the
      valid-subaperture counts uneven.
    * DMs: 81^2 / 47^2 / 37^2 Fried grids spanning 480 px on 512^2 IF grids at the
      pupil pixel scale, actuators within one pitch of the 240-px radius kept.
    * Pair (w, d): cone scale 1 - h/H, footprint centre h*alpha along the LGS azimuth.
    """
    rng = rng_for(seed)
    D = 39.0
    n_px = n_sub * p
    pix = D / n_px
    H = 90e3
    alpha = math.radians(45.0 / 3600.0)
    alts = [0.0, 4e3, 12.7e3]
    n1d = [81, 47, 37]
    az = [math.radians(60.0 * w) for w in range(n_wfs)]
    pupils, valids, clock = [], [], []
    for w in range(n_wfs):
        off = (float(rng.uniform(-p / 2, p / 2)), float(rng.uniform(-p / 2, p / 2)))
        P = pupil_mask(n_px, float(n_px), 0.28, off)
        pupils.append(P)
        valids.append(valid_subapertures(P, p))
        rot = math.degrees(az[w]) % 90.0 - 45.0
        clock.append((math.radians(rot), off))
    grids = []
    for n in n1d:
        pitch = 480.0 / (n - 1)
        grids.append(actuator_grid(n, pitch, 512, keep_radius=240.0 + pitch))
    pairs = []
    for w in range(n_wfs):
        rot, off = clock[w]
        for d, h in enumerate(alts):
            f = h * alpha / pix
            g = Geometry(cone_scale=1.0 - h / H,
                         footprint_x=f * math.cos(az[w]), footprint_y=f * math.sin(az[w]),
                         wfs_rot=rot, wfs_shift_x=off[0], wfs_shift_y=off[1])
            pairs.append(McaoPair(w, d, g))
    return McaoConfig(n_sub, p, pupils, valids, grids, alts, pairs, pix, H, alpha, az)


# ------------------------------------------------------- probes and learned-fit data
def _noll_to_nm(j: int) -> Tuple[int, int]:
    """Noll index j >= 1 -> (n, m) with signed azimuthal order m."""
    n = 0
    while (n + 1) * (n + 2) // 2 < j:
        n += 1
    k = j - n * (n + 1) // 2 - 1          # 0-based position within radial order n
    ms = [m for m in range(n % 2, n + 1, 2)]
    # position k covers |m| values in increasing order, two entries per m>0
    order = []
    for m in ms:
        order.extend([m] if m == 0 else [m, m])
    am = order[k]
    if am == 0:
        return n, 0
    return n, (am if j % 2 == 0 else -am)


def zernike_noll(j: int, n_px: int, diameter: float) -> np.ndarray:
    """Noll-normalised Zernike Z_j sampled at pixel centres of an n_px grid (float64).

    Normalised to unit RMS over the unit disk; values outside the disk are zero.
    """
    n, m = _noll_to_nm(j)
    c = (n_px - 1) / 2.0
    y, x = np.mgrid[0:n_px, 0:n_px].astype(np.float64)
    X = (x - c) / (diameter / 2.0)
    Y = (y - c) / (diameter / 2.0)
    r = np.hypot(X, Y)
    t = np.arctan2(Y, X)
    am = abs(m)
    R = np.zeros_like(r)
    for s in range((n - am) // 2 + 1):
        coef = ((-1) ** s * math.factorial(n - s)
                / (math.factorial(s) * math.factorial((n + am) // 2 - s) * math.factorial((n - am) // 2 - s)))
        R += coef * r ** (n - 2 * s)
    if m == 0:
        Z = math.sqrt(n + 1) * R
    elif m > 0:
        Z = math.sqrt(2 * (n + 1)) * R * np.cos(am * t)
    else:
        Z = math.sqrt(2 * (n + 1)) * R * np.sin(am * t)
    Z[r > 1.0] = 0.0
    return Z


def probe_commands(grid: ActuatorGrid, pupil_on_if: np.ndarray, modes: Sequence[int],
                   diameter: Optional[float] = None) -> np.ndarray:
    """Least-squares actuator commands C [n_act][n_modes] fitting each Zernike.

    Fit is over the nominal pupil pixels on the IF grid (``pupil_on_if`` is a
    boolean mask on that grid); Zernikes are defined on that same pupil.
    """
    ifs = if_stack(grid).astype(np.float64)
    sel = pupil_on_if.astype(bool)
    Amat = ifs[:, sel].T                                  # [n_pix][n_act]
    n = grid.grid_n
    diam = float(diameter) if diameter is not None else 2.0 * math.sqrt(sel.sum() / math.pi)
    Z = np.stack([zernike_noll(j, n, diam)[sel] for j in modes], axis=1)
    C, *_ = np.linalg.lstsq(Amat, Z, rcond=None)
    return C


@dataclass
class ProbeConfig:
    """Learned-misregistration workload: cfg-1 WFS, 9x9 DM on an enlarged 128^2 IF grid."""
    scao: ScaoConfig
    modes: Tuple[int, ...]
    commands: np.ndarray        # float64 [81][20]
    probe_maps: np.ndarray      # float32 [20][128][128] = sum_a C[a,j] IF_a
    feat_len: int = 4000


def probe_config() -> ProbeConfig:
    base = scao_small()
    grid = actuator_grid(9, 10.0, 128)
    scao = ScaoConfig("scao_8x8_probe", base.n_sub, base.p, base.pupil, base.valid, grid, base.theta)
    c = (128 - 1) / 2.0
    yy, xx = np.mgrid[0:128, 0:128].astype(np.float64)
    on_if = np.hypot(xx - c, yy - c) <= 40.0
    modes = tuple(range(2, 22))
    C = probe_commands(grid, on_if, modes, diameter=80.0)
    ifs = if_stack(grid).astype(np.float64)
    maps = np.einsum("aj,ayx->jyx", C, ifs).astype(np.float32)
    return ProbeConfig(scao, modes, C, maps)


LABEL_LO = np.array([-10.0, -10.0, math.radians(-1.0), 0.98])
LABEL_HI = np.array([10.0, 10.0, math.radians(1.0), 1.02])


def draw_misreg_labels(seed: int, p: int = 10):
    """One learned-fit sample: theta (shift U(-1,1) subaperture = U(-p,p) px,
    rotation U(-1,1) deg, magnification U(0.98,1.02)), an SNR U(20,200) and
    the seed's standard-normal noise generator state.
    Returns (theta float64[4], snr, rng) with rng positioned after the draws.
    """
    rng = rng_for(seed)
    tx = rng.uniform(-1.0, 1.0) * p
    ty = rng.uniform(-1.0, 1.0) * p
    rot = math.radians(rng.uniform(-1.0, 1.0))
    mag = rng.uniform(0.98, 1.02)
    snr = rng.uniform(20.0, 200.0)
    return np.array([tx, ty, rot, mag]), float(snr), rng


# ------------------------------------------------------------ modal basis (Fourier)
@dataclass
class FourierMode:
    """cos or sin of 2 pi (kx x + ky y) / period on the IF grid, about centre c."""
    kx: int
    ky: int
    kind: int                   # 0: cos, 1: sin


def fourier_modes(n_modes: int) -> List[FourierMode]:
    """The first n_modes of a Fourier modal basis, ordered by spatial frequency:
    frequency vectors (kx, ky) of the half plane (ky > 0, or ky = 0 and kx > 0),
    by |k| then angle, each giving a cos and a sin mode.  The piston is left out.
    A synthetic stand-in for the modal stacks (KL, Zernike, M4 modes) a DM can be
    driven with: dense maps over the whole grid whose high orders carry the
    spatial frequencies an interpolation filters."""
    ks = []
    r = 1
    while len(ks) * 2 < n_modes:
        ks = [(kx, ky) for ky in range(0, r + 1) for kx in range(-r, r + 1)
              if (ky > 0 or kx > 0) and kx * kx + ky * ky <= r * r]
        r += 1
    ks.sort(key=lambda k: (k[0] * k[0] + k[1] * k[1], math.atan2(k[1], k[0])))
    out = []
    for kx, ky in ks:
        out.append(FourierMode(kx, ky, 0))
        out.append(FourierMode(kx, ky, 1))
    return out[:n_modes]


def fourier_mode_values(mode: FourierMode, x, y, period: float, cx: float, cy: float):
    """The mode's exact value at arbitrary points (float64 arrays x, y)."""
    ph = 2.0 * math.pi * (mode.kx * (np.asarray(x, np.float64) - cx) +
                          mode.ky * (np.asarray(y, np.float64) - cy)) / period
    return np.cos(ph) if mode.kind == 0 else np.sin(ph)


def fourier_stack(modes: Sequence[FourierMode], grid_n: int, period: float) -> np.ndarray:
    """float32 [M][grid_n][grid_n]: every mode at the IF pixel centres, about the
    grid centre."""
    c = (grid_n - 1) / 2.0
    yy, xx = np.mgrid[0:grid_n, 0:grid_n].astype(np.float64)
    return np.stack([fourier_mode_values(m, xx, yy, period, c, c) for m in modes]).astype(
        np.float32)


def fourier_stack_torch(modes: Sequence[FourierMode], grid_n: int, period: float, device,
                        chunk: int = 256):
    """fourier_stack built on a torch device in float64 chunks, rounded to float32."""
    import torch
    c = (grid_n - 1) / 2.0
    t = torch.arange(grid_n, dtype=torch.float64, device=device) - c
    kx = torch.tensor([m.kx for m in modes], dtype=torch.float64, device=device)
    ky = torch.tensor([m.ky for m in modes], dtype=torch.float64, device=device)
    kind = torch.tensor([m.kind for m in modes], dtype=torch.bool, device=device)
    out = torch.empty((len(modes), grid_n, grid_n), dtype=torch.float32, device=device)
    w = 2.0 * math.pi / period
    for a0 in range(0, len(modes), chunk):
        a1 = min(len(modes), a0 + chunk)
        ph = w * (kx[a0:a1, None, None] * t[None, None, :] + ky[a0:a1, None, None] * t[None, :, None])
        v = torch.where(kind[a0:a1, None, None], torch.sin(ph), torch.cos(ph))
        out[a0:a1] = v.to(torch.float32)
        del ph, v
    return out
