"""Object, PSF and noise generators (see the package docstring)."""
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import zlib

import numpy as np


def stable_seed(*parts) -> int:
    """A 32-bit seed from the repr of `parts` (CRC-32): the same on every run
    and in every process, unlike hash(), which randomises strings."""
    return zlib.crc32(repr(parts).encode())


@dataclass(frozen=True)
class VolumeConfig:
    name: str
    shape: Tuple[int, ...]          # X extent m, (z, y, x) or (y, x)
    psf_shape: Tuple[int, ...]      # 2p+1 per axis
    sigmas: Tuple[float, ...]       # Gaussian sigma per axis (voxels)
    seed: int
    n_points: int
    n_filaments: int = 0
    n_blobs: int = 0
    point_amp: Tuple[float, float] = (0.2, 1.0)
    background: float = 0.01
    peak_photons: float = 500.0
    read_noise: float = 2.0
    dtype: str = "float32"
    iters: int = 100
    extra: dict = field(default_factory=dict)


CONFIGS = {
    # 2-D, FP64: 64x64 X, 9x9 PSF sigma 1.5, Poisson at peak 1000, 50 iterations.
    "c1_2d_f64": VolumeConfig("c1_2d_f64", (64, 64), (9, 9), (1.5, 1.5), seed=0, n_points=40, n_blobs=5,
                              point_amp=(0.5, 1.0), peak_photons=1000.0, read_noise=0.0,
                              dtype="float64", iters=50),
    # 3-D, FP32: 128x128x64 X, 15x15x31 PSF (sigma_xy 2, sigma_z 5), 100 iterations.
    "c2_3d_f32": VolumeConfig("c2_3d_f32", (64, 128, 128), (31, 15, 15), (5.0, 2.0, 2.0), seed=1,
                              n_points=500, n_filaments=30, iters=100),
    # 3-D precision/metric workload: 512x512x128 X, 31x31x63 PSF (sigma_xy 3, sigma_z 9).
    "c3_metric": VolumeConfig("c3_metric", (128, 512, 512), (63, 31, 31), (9.0, 3.0, 3.0), seed=2,
                              n_points=8000, n_filaments=400, iters=100),
    # Differentiable workload: 256x256x64 X, true PSF 21x21x41 (sigma_xy 2.5, sigma_z 6).
    "c5_diff": VolumeConfig("c5_diff", (64, 256, 256), (41, 21, 21), (6.0, 2.5, 2.5), seed=4,
                            n_points=2000, n_filaments=100, iters=20,
                            extra={"guess_sigmas": (5.0, 2.0, 2.0)}),
}

# Small-PSF (HBM-bound) sweep on the metric volume.
SWEEP_PSFS = {3: (0.8, 0.8, 0.8), 5: (1.2, 1.2, 1.2), 7: (1.6, 1.6, 1.6)}


def gaussian_factors(psf_shape: Sequence[int], sigmas: Sequence[float]) -> List[np.ndarray]:
    """1-D factors f_i(t) = exp(-t^2 / (2 sigma_i^2)) on t in [-p_i, p_i],
    each normalised to sum 1; their outer product is the normalised PSF."""
    out = []
    for e, s in zip(psf_shape, sigmas):
        if e % 2 != 1:
            raise ValueError("PSF extents must be odd")
        p = (e - 1) // 2
        t = np.arange(-p, p + 1, dtype=np.float64)
        f = np.exp(-(t * t) / (2.0 * s * s))
        out.append(f / f.sum())
    return out


def gaussian_psf(psf_shape: Sequence[int], sigmas: Sequence[float]) -> np.ndarray:
    """h(t) proportional to exp(-sum_i t_i^2 / (2 sigma_i^2)), sampled at
    integer offsets from the centre and normalised to sum 1 (float64)."""
    fs = gaussian_factors(psf_shape, sigmas)
    h = fs[0]
    for f in fs[1:]:
        h = np.multiply.outer(h, f)
    return h / h.sum()


def _render_points(vol, rng, n, amp):
    idx = tuple(rng.integers(0, e, size=n) for e in vol.shape)
    a = rng.uniform(amp[0], amp[1], size=n)
    np.maximum.at(vol, idx, a)


def _render_blobs(vol, rng, n):
    grids = np.meshgrid(*[np.arange(e, dtype=np.float64) for e in vol.shape], indexing="ij")
    for _ in range(n):
        c = [rng.uniform(0, e - 1) for e in vol.shape]
        s = rng.uniform(1.0, 3.0)
        a = rng.uniform(0.5, 1.0)
        d2 = sum((g - ci) ** 2 for g, ci in zip(grids, c))
        np.maximum(vol, a * np.exp(-d2 / (2 * s * s)), out=vol)


def _render_filaments(vol, rng, n):
    """Quadratic Bezier curves with uniform end and control points, sampled
    every 0.25 voxel; every voxel within the tube radius U[1,2] of a sample
    takes max(current, intensity U[0.2,1])."""
    shape = np.array(vol.shape)
    nd = len(shape)
    for _ in range(n):
        P = rng.uniform(0, 1, size=(3, nd)) * (shape - 1)
        r = rng.uniform(1.0, 2.0)
        inten = rng.uniform(0.2, 1.0)
        length = np.linalg.norm(P[1] - P[0]) + np.linalg.norm(P[2] - P[1])
        ns = max(2, int(np.ceil(length / 0.25)) + 1)
        t = np.linspace(0.0, 1.0, ns)[:, None]
        pts = (1 - t) ** 2 * P[0] + 2 * (1 - t) * t * P[1] + t ** 2 * P[2]
        R = int(np.ceil(r))
        off = np.stack(np.meshgrid(*[np.arange(-R, R + 1)] * nd, indexing="ij"), -1).reshape(-1, nd)
        base = np.rint(pts).astype(np.int64)
        cand = (base[:, None, :] + off[None, :, :]).reshape(-1, nd)
        d2 = np.sum((cand - np.repeat(pts, len(off), axis=0)) ** 2, axis=1)
        keep = (d2 <= r * r) & np.all((cand >= 0) & (cand < shape), axis=1)
        flat = np.ravel_multi_index(tuple(cand[keep].T), vol.shape)
        v = vol.reshape(-1)
        # duplicates all write max(old, inten) of the same old value
        v[flat] = np.maximum(v[flat], inten)


def make_objects(cfg: VolumeConfig, shape: Optional[Tuple[int, ...]] = None,
                 rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """Non-negative ground-truth object X (float64) for a config."""
    shape = tuple(shape or cfg.shape)
    rng = rng or np.random.default_rng(cfg.seed)
    vol = np.full(shape, cfg.background, dtype=np.float64)
    _render_points(vol, rng, cfg.n_points, cfg.point_amp)
    if cfg.n_blobs:
        _render_blobs(vol, rng, cfg.n_blobs)
    if cfg.n_filaments:
        _render_filaments(vol, rng, cfg.n_filaments)
    return vol


def psf_for(cfg: VolumeConfig) -> np.ndarray:
    return gaussian_psf(cfg.psf_shape, cfg.sigmas)


def add_noise(blurred: np.ndarray, cfg: VolumeConfig, rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """Scale the blurred image so its maximum is cfg.peak_photons, draw
    Poisson counts, then add N(0, read_noise^2) read noise (Y may go
    negative).  Returned in photon units, float64."""
    rng = rng or np.random.default_rng(cfg.seed + 1000)
    b = np.asarray(blurred, dtype=np.float64)
    scale = cfg.peak_photons / max(float(b.max()), 1e-30)
    y = rng.poisson(np.maximum(b * scale, 0.0)).astype(np.float64)
    if cfg.read_noise > 0:
        y += rng.normal(0.0, cfg.read_noise, size=y.shape)
    return y


def flat_start(y: np.ndarray, h: np.ndarray, x_shape: Sequence[int]) -> np.ndarray:
    """Flux-matching flat initial solution X^0 = max(sum Y, 0)/(N sum H)."""
    n = int(np.prod(x_shape))
    v = max(float(np.sum(y)), 0.0) / (n * float(np.sum(h)))
    return np.full(tuple(x_shape), v, dtype=np.float64)


def batched_configs(count: int = 64, seed: int = 3) -> List[VolumeConfig]:
    """Independent volumes for the batched workload: z ~ U{32..96},
    y, x ~ U{32..160}; each PSF has odd extent U{9,11,..,31} per axis and
    sigma_z, sigma_xy ~ U[1,6]; structure density scaled to the volume."""
    rng = np.random.default_rng(seed)
    out = []
    ref_vox = 64 * 128 * 128
    for i in range(count):
        shape = (int(rng.integers(32, 97)), int(rng.integers(32, 161)), int(rng.integers(32, 161)))
        psf = tuple(int(2 * rng.integers(4, 16) + 1) for _ in range(3))
        sz, sxy = float(rng.uniform(1, 6)), float(rng.uniform(1, 6))
        frac = np.prod(shape) / ref_vox
        out.append(VolumeConfig("c4_vol%02d" % i, shape, psf, (sz, sxy, sxy), seed=seed * 1000 + i,
                                n_points=max(1, int(500 * frac)), n_filaments=max(1, int(30 * frac)),
                                iters=50))
    return out


# ---- 2-D stand-ins for the paper's two experiments (its images are not
# available): a 512x512 phantom of nine crossing lines, and a 225x225 8-bit
# piecewise-smooth image blurred by a 5x5 PSF; both get additive Gaussian
# white noise of a stated standard deviation.

def crossing_lines(shape: Tuple[int, int] = (512, 512), n: int = 9, width: float = 3.0, amp: float = 255.0,
                   seed: int = 7) -> np.ndarray:
    """n straight lines across the image at distinct angles, each through a
    point of the central half, `width` pixels wide with a one-pixel linear
    edge, value amp on a zero background (max at crossings)."""
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.arange(shape[0], dtype=np.float64), np.arange(shape[1], dtype=np.float64),
                         indexing="ij")
    img = np.zeros(shape, dtype=np.float64)
    angles = np.pi * (np.arange(n) + rng.uniform(0.1, 0.9, size=n)) / n
    for a in angles:
        cy, cx = rng.uniform(0.25, 0.75) * (shape[0] - 1), rng.uniform(0.25, 0.75) * (shape[1] - 1)
        d = np.abs(-(yy - cy) * np.cos(a) + (xx - cx) * np.sin(a))   # distance to the line
        np.maximum(img, amp * np.clip(width / 2 + 0.5 - d, 0.0, 1.0), out=img)
    return img


def piecewise_image(shape: Tuple[int, int] = (225, 225), seed: int = 8) -> np.ndarray:
    """8-bit-range piecewise-smooth image: a shaded background, 12 ellipses
    and 6 rectangles of random grey levels, 20 small bright spots; clipped to
    [0, 255]."""
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.arange(shape[0], dtype=np.float64), np.arange(shape[1], dtype=np.float64),
                         indexing="ij")
    img = 40.0 + 60.0 * (yy / shape[0]) + 30.0 * (xx / shape[1])
    for _ in range(12):
        cy, cx = rng.uniform(0, shape[0]), rng.uniform(0, shape[1])
        ry, rx = rng.uniform(6, 40), rng.uniform(6, 40)
        th = rng.uniform(0, np.pi)
        u = ((yy - cy) * np.cos(th) + (xx - cx) * np.sin(th)) / ry
        v = (-(yy - cy) * np.sin(th) + (xx - cx) * np.cos(th)) / rx
        img[u * u + v * v <= 1.0] = rng.uniform(0, 255)
    for _ in range(6):
        y0, x0 = rng.integers(0, shape[0] - 20), rng.integers(0, shape[1] - 20)
        h, w = rng.integers(8, 40), rng.integers(8, 40)
        img[y0:y0 + h, x0:x0 + w] = rng.uniform(0, 255)
    for _ in range(20):
        cy, cx = rng.uniform(0, shape[0]), rng.uniform(0, shape[1])
        img = np.maximum(img, 255.0 * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * 1.5 ** 2)))
    return np.clip(img, 0.0, 255.0)


def gaussian_noise(blurred: np.ndarray, std: float, seed: int) -> np.ndarray:
    """Y = blurred + N(0, std^2) white noise (float64)."""
    rng = np.random.default_rng(seed)
    b = np.asarray(blurred, dtype=np.float64)
    return b + rng.normal(0.0, std, size=b.shape)


# The two paper-shape workloads: (object, PSF extent, PSF sigma, noise std list).
PAPER_2D = {
    # Fig. 1 stand-in: 512x512, nine crossing lines; the paper gives no PSF:
    # a 9x9 Gaussian, sigma 2, is used; noise std 5.
    "lines512": {"object": lambda: crossing_lines(), "psf": (9, 9), "sigma": (2.0, 2.0), "noise": (5.0,)},
    # Fig. 2 stand-in: 225x225 8-bit image, 5x5 PSF (a Gaussian, sigma 1),
    # noise std 20 and 5.
    "image225": {"object": lambda: piecewise_image(), "psf": (5, 5), "sigma": (1.0, 1.0), "noise": (20.0, 5.0)},
}
