"""Seeded synthetic inputs for the DBIE hot path: boundary magnetograms, evaluation points and lambda.

This module holds input recipes only (no DBIE arithmetic). Both the CPU oracle and the GPU path take
their inputs from here. Every recipe is deterministic for its seed: numpy default_rng with
SeedSequence sub-streams.

Units: lengths are in pixels unless a workload states otherwise; the pixel (a, b) centre is
(x0 + a*h, y0 + b*h, 0). B0 has shape [3, ny, nx] (component-major, x fastest). Points have shape
[3, N] (x, y, z rows). lambda has shape [3, N] (one pseudo-force-free factor per field component and
point, Section 2.1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .lowlou import LowLou


@dataclass
class Boundary:
    B0: np.ndarray            # [3, ny, nx] float64 (FP32-representable where the workload is FP32)
    x0: float = 0.0
    y0: float = 0.0
    h: float = 1.0

    @property
    def nx(self) -> int:
        return int(self.B0.shape[2])

    @property
    def ny(self) -> int:
        return int(self.B0.shape[1])


@dataclass
class Workload:
    name: str
    boundaries: List[Boundary]
    xyz: np.ndarray                       # [3, N] float64
    seg: np.ndarray                       # [n_boundaries + 1] int64 point offsets
    lam: Optional[np.ndarray] = None      # [3, N] float64 throughput lambda (None: solve from 0)
    fp32: bool = True                     # the boundary data were rounded to FP32 once
    meta: dict = field(default_factory=dict)

    @property
    def n_points(self) -> int:
        return int(self.xyz.shape[1])

    def pairs_per_trial(self) -> int:
        tot = 0
        for b, bd in enumerate(self.boundaries):
            tot += bd.nx * bd.ny * int(self.seg[b + 1] - self.seg[b])
        return int(tot)


def _rngs(seed: int, n: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


# ------------------------------------------------------------------------------------------------
# magnetogram pieces
# ------------------------------------------------------------------------------------------------
def gaussian_bipoles(nx: int, ny: int, nbip: int, rng, sigma_range=(3.0, 12.0),
                     amp_range=(500.0, 2500.0), sigma_cap: Optional[float] = None,
                     margin_sigmas: float = 3.0):
    """List of flux-balanced Gaussian bipoles (sigma, amplitude, pole centres) inside the frame.

    Pole separation is U[2 sigma, 4 sigma] at a uniform random angle; both poles keep at least
    margin_sigmas * sigma from the edges (the separation shrinks when the frame is too small).
    """
    out = []
    for _ in range(nbip):
        s = rng.uniform(*sigma_range)
        if sigma_cap is not None:
            s = min(s, sigma_cap)
        A = rng.uniform(*amp_range)
        sep = rng.uniform(2.0 * s, 4.0 * s)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        m = margin_sigmas * s
        room_x = (nx - 1) - 2 * m
        room_y = (ny - 1) - 2 * m
        dx = 0.5 * sep * np.cos(ang)
        dy = 0.5 * sep * np.sin(ang)
        # shrink the separation to fit
        scale = 1.0
        if 2 * abs(dx) > room_x:
            scale = min(scale, room_x / (2 * abs(dx) + 1e-300))
        if 2 * abs(dy) > room_y:
            scale = min(scale, room_y / (2 * abs(dy) + 1e-300))
        dx *= max(scale, 0.0)
        dy *= max(scale, 0.0)
        cx = rng.uniform(m + abs(dx), (nx - 1) - m - abs(dx))
        cy = rng.uniform(m + abs(dy), (ny - 1) - m - abs(dy))
        out.append(dict(sigma=s, A=A, p=(cx + dx, cy + dy), n=(cx - dx, cy - dy)))
    return out


def bipole_bz(nx: int, ny: int, bip) -> np.ndarray:
    X, Y = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64))
    s2 = 2.0 * bip["sigma"] ** 2
    gp = np.exp(-((X - bip["p"][0]) ** 2 + (Y - bip["p"][1]) ** 2) / s2)
    gn = np.exp(-((X - bip["n"][0]) ** 2 + (Y - bip["n"][1]) ** 2) / s2)
    return bip["A"] * (gp - gn)


def potential_psi(Bz: np.ndarray) -> np.ndarray:
    """Scalar potential at z=0 of the potential field with normal component Bz (psi_hat = Bz_hat/|k|,
    zero mean), computed by FFT on a 2x zero-padded grid."""
    ny, nx = Bz.shape
    P = np.zeros((2 * ny, 2 * nx))
    P[:ny, :nx] = Bz
    F = np.fft.rfft2(P)
    ky = 2 * np.pi * np.fft.fftfreq(2 * ny)
    kx = 2 * np.pi * np.fft.rfftfreq(2 * nx)
    K = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    K[0, 0] = 1.0
    F = F / K
    F[0, 0] = 0.0
    return np.fft.irfft2(F, s=P.shape)[:ny, :nx]


def sheared_horizontal(psi: np.ndarray, alpha: float):
    """(Bx, By) = alpha * (d psi/dy, d psi/dx) by centred differences (one-sided at the edges)."""
    dpsi_dy, dpsi_dx = np.gradient(psi)
    return alpha * dpsi_dy, alpha * dpsi_dx


def bipole_magnetogram(nx, ny, nbip, rng_layout, rng_noise, alpha_range=(1.0, 1.0),
                       sigma_range=(3.0, 12.0), amp_range=(500.0, 2500.0), sigma_cap=None,
                       noise_sigma=20.0):
    bips = gaussian_bipoles(nx, ny, nbip, rng_layout, sigma_range, amp_range, sigma_cap)
    B = np.zeros((3, ny, nx))
    for bip in bips:
        bz = bipole_bz(nx, ny, bip)
        alpha = rng_layout.uniform(*alpha_range)
        bx, by = sheared_horizontal(potential_psi(bz), alpha)
        B[0] += bx
        B[1] += by
        B[2] += bz
        bip["alpha"] = alpha
    if noise_sigma > 0:
        B[0] += rng_noise.normal(0.0, noise_sigma, size=(ny, nx))
        B[1] += rng_noise.normal(0.0, noise_sigma, size=(ny, nx))
    return B, bips


def to_fp32_once(B: np.ndarray) -> np.ndarray:
    return B.astype(np.float32).astype(np.float64)


def grid_points(nx, ny, nz, x0=0.0, y0=0.0, h=1.0, zstep=1.0):
    """Points above pixel centres, z = k*zstep*h for k = 1..nz; ordered (z, y, x) with x fastest."""
    z, y, x = np.meshgrid(np.arange(1, nz + 1) * zstep * h, y0 + h * np.arange(ny),
                          x0 + h * np.arange(nx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()])


def z_stratified_subsample(xyz: np.ndarray, n_sub: int, seed: int) -> np.ndarray:
    """Indices of a seeded subsample with the same number of points on every z level; with more
    distinct heights than n_sub (continuous z), one point from each of n_sub equal-count bins of z."""
    rng = np.random.default_rng(seed)
    levels = np.unique(xyz[2])
    if len(levels) > n_sub:
        order = np.argsort(xyz[2], kind="stable")
        edges = np.linspace(0, order.size, n_sub + 1).astype(np.int64)   # n_sub bins of equal count
        pick = edges[:-1] + (rng.random(n_sub) * (edges[1:] - edges[:-1])).astype(np.int64)
        return np.sort(order[pick])
    per = max(1, n_sub // len(levels))
    idx = []
    for zl in levels:
        cand = np.nonzero(xyz[2] == zl)[0]
        idx.append(np.sort(rng.choice(cand, size=min(per, cand.size), replace=False)))
    return np.concatenate(idx)


# ------------------------------------------------------------------------------------------------
# the five workloads
# ------------------------------------------------------------------------------------------------
_LL_CACHE = {}


def lowlou_case(n=1, m=1, l=0.3, Phi=np.pi / 4) -> LowLou:
    key = (n, m, l, Phi)
    if key not in _LL_CACHE:
        _LL_CACHE[key] = LowLou(n=n, m=m, l=l, Phi=Phi)
    return _LL_CACHE[key]


def config1(seed: int = 1001) -> Workload:
    """Low & Lou n=1, m=1, l=0.3, Phi=pi/4 on a 32x32 FP64 cell-centred grid over [-1,1]^2
    (h = 1/16) and an 8x8x8 interior grid x,y = -1+(j+1/2)/4, z = k/8."""
    ll = lowlou_case()
    h = 1.0 / 16.0
    x0 = -1.0 + 0.5 * h
    xs = x0 + h * np.arange(32)
    X, Y = np.meshgrid(xs, xs)
    B0 = ll.field(X, Y, np.zeros_like(X))
    pz, py, px = np.meshgrid(np.arange(1, 9) / 8.0, -1.0 + (np.arange(8) + 0.5) / 4.0,
                             -1.0 + (np.arange(8) + 0.5) / 4.0, indexing="ij")
    xyz = np.stack([px.ravel(), py.ravel(), pz.ravel()])
    rng = np.random.default_rng(seed)
    lam = rng.uniform(-2.0, 2.0, size=(3, xyz.shape[1]))
    return Workload("lowlou_32x32_8x8x8", [Boundary(B0, x0, x0, h)], xyz,
                    np.array([0, xyz.shape[1]], np.int64), lam, fp32=False,
                    meta=dict(ll=ll, nm_budget=50, eps=1e-4))


def config2(seed: int = 1002, nz: int = 64) -> Workload:
    """128x128 FP32 magnetogram of 6 Gaussian bipoles with sheared horizontal field (alpha = 1)
    plus N(0, 20 G) noise; points on the 128x128x64 grid; throughput lambda ~ U(-4pi/128, 4pi/128)."""
    r_layout, r_noise, r_lam = _rngs(seed, 3)
    B0, bips = bipole_magnetogram(128, 128, 6, r_layout, r_noise, alpha_range=(1.0, 1.0))
    B0 = to_fp32_once(B0)
    xyz = grid_points(128, 128, nz)
    lm = 4.0 * np.pi / 128.0
    lam = r_lam.uniform(-lm, lm, size=xyz.shape)
    return Workload("bipoles_128x128_128x128x%d" % nz, [Boundary(B0)], xyz,
                    np.array([0, xyz.shape[1]], np.int64), lam, meta=dict(bipoles=bips))


def config3(seed: int = 1003, nxy: int = 256, nz: int = 128) -> Workload:
    """256x256 FP32 magnetogram of 10 bipoles with per-bipole shear alpha ~ U[0.5, 2]; points on
    the 256x256x128 grid; lambda solved from 0."""
    r_layout, r_noise, r_lam = _rngs(seed, 3)
    B0, bips = bipole_magnetogram(nxy, nxy, 10, r_layout, r_noise, alpha_range=(0.5, 2.0))
    B0 = to_fp32_once(B0)
    xyz = grid_points(nxy, nxy, nz)
    lm = 4.0 * np.pi / nxy
    lam = r_lam.uniform(-lm, lm, size=xyz.shape)
    return Workload("bipoles_%dx%d_%dx%dx%d" % (nxy, nxy, nxy, nxy, nz), [Boundary(B0)], xyz,
                    np.array([0, xyz.shape[1]], np.int64), lam, meta=dict(bipoles=bips))


def config4(seed: int = 1004, n_mag: int = 64, npts_range=(2 ** 14, 2 ** 17),
            side_range=(64, 192)) -> Workload:
    """64 independent magnetograms (side U{64..192}, 2-8 bipoles with sigma <= side/10, alpha ~
    U[0.5,2]), each with U{2^14..2^17} random points x,y ~ U(-0.5, side-0.5), z ~ U(0.5, 64)."""
    rngs = _rngs(seed, 4 * n_mag)
    bds, pts, lams, seg = [], [], [], [0]
    for b in range(n_mag):
        r_size, r_layout, r_noise, r_pts = rngs[4 * b: 4 * b + 4]
        side = int(r_size.integers(side_range[0], side_range[1] + 1))
        nbip = int(r_size.integers(2, 9))
        npts = int(r_size.integers(npts_range[0], npts_range[1] + 1))
        B0, _ = bipole_magnetogram(side, side, nbip, r_layout, r_noise, alpha_range=(0.5, 2.0),
                                   sigma_cap=side / 10.0)
        bds.append(Boundary(to_fp32_once(B0)))
        x = r_pts.uniform(-0.5, side - 0.5, npts)
        y = r_pts.uniform(-0.5, side - 0.5, npts)
        z = r_pts.uniform(0.5, 64.0, npts)
        pts.append(np.stack([x, y, z]))
        lm = 4.0 * np.pi / side
        lams.append(r_pts.uniform(-lm, lm, size=(3, npts)))
        seg.append(seg[-1] + npts)
    return Workload("batched_%d_magnetograms" % n_mag, bds, np.concatenate(pts, axis=1),
                    np.array(seg, np.int64), np.concatenate(lams, axis=1))


def config5(seed: int = 1005, n_arcs: int = 4096, per_arc: int = 256) -> Workload:
    """512x256 FP32 active-region-like magnetogram: 20 bipoles plus one strongly sheared pair
    (A = 3000 G, sigma = 8, alpha = 3) on a common inversion line, rescaled to max|B| = 3000 G;
    points clustered on n_arcs semicircular arcs between opposite-polarity footpoints."""
    r_layout, r_noise, r_arc, r_lam = _rngs(seed, 4)
    nx, ny = 512, 256
    B0, bips = bipole_magnetogram(nx, ny, 20, r_layout, r_noise, alpha_range=(0.5, 2.0))
    core = dict(sigma=8.0, A=3000.0, p=(nx / 2 - 12.0, ny / 2), n=(nx / 2 + 12.0, ny / 2))
    bz = bipole_bz(nx, ny, core)
    bx, by = sheared_horizontal(potential_psi(bz), 3.0)
    B0[0] += bx
    B0[1] += by
    B0[2] += bz
    B0 *= 3000.0 / np.max(np.sqrt(np.sum(B0 * B0, axis=0)))
    B0 = to_fp32_once(B0)
    bz = B0[2]
    pos = np.maximum(bz, 0).ravel()
    neg = np.maximum(-bz, 0).ravel()
    X, Y = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64))
    X = X.ravel()
    Y = Y.ravel()
    ia = r_arc.choice(nx * ny, size=n_arcs, p=pos / pos.sum())
    pts = []
    s = (np.arange(per_arc) + 0.5) / per_arc
    for a in ia:
        near = (X - X[a]) ** 2 + (Y - Y[a]) ** 2 <= 128.0 ** 2
        w = neg * near
        if w.sum() <= 0:
            w = neg
        ib = r_arc.choice(nx * ny, p=w / w.sum())
        A = np.array([X[a], Y[a]])
        Bp = np.array([X[ib], Y[ib]])
        hor = A[:, None] + (Bp - A)[:, None] * s[None, :]
        z = np.maximum(0.5, 0.5 * np.linalg.norm(Bp - A) * np.sin(np.pi * s))
        pts.append(np.vstack([hor, z[None, :]]))
    xyz = np.concatenate(pts, axis=1)
    lm = 4.0 * np.pi / nx
    lam = r_lam.uniform(-lm, lm, size=xyz.shape)
    return Workload("active_region_512x256_arcs", [Boundary(B0)], xyz,
                    np.array([0, xyz.shape[1]], np.int64), lam, meta=dict(bipoles=bips))


def lowlou_table1(seed: int = 1006, mapping: str = "region") -> Workload:
    """The Table 1 comparison case: Low & Lou n=3, m=1, l=0.3, Phi=4pi/5 sampled on a 192x192 pixel
    lower boundary centred on a 64x64x64-pixel test region. The case's own grid definition is not
    reproduced in the paper; two mappings are offered: mapping="region", the test region spans
    [-1, 1]^2 x [0, 2] (h = 1/32, the boundary [-3, 3]^2); mapping="boundary", the boundary spans
    [-1, 1]^2 (h = 1/96, the region [-1/3, 1/3]^2 x [0, 2/3]). Boundary nodes at ((k - 95.5) h,
    (j - 95.5) h); region nodes at x, y = (i - 31.5) h (the central 64 x 64 boundary nodes) and
    z = k h, k = 0..63. The points are the layers k >= 1 (z > 0); the k = 0 layer is the boundary
    data itself (meta['bottom_idx'] are its pixels)."""
    ll = lowlou_case(n=3, m=1, l=0.3, Phi=4.0 * np.pi / 5.0)
    h = {"region": 1.0 / 32.0, "boundary": 2.0 / 192.0}[mapping]
    x0 = -95.5 * h
    xs = x0 + h * np.arange(192)
    X, Y = np.meshgrid(xs, xs)
    B0 = ll.field(X, Y, np.zeros_like(X))
    rs = (np.arange(64) - 31.5) * h
    pz, py, px = np.meshgrid(h * np.arange(1, 64), rs, rs, indexing="ij")
    xyz = np.stack([px.ravel(), py.ravel(), pz.ravel()])
    rng = np.random.default_rng(seed)
    lam = rng.uniform(-2.0, 2.0, size=(3, xyz.shape[1]))
    jj, ii = np.meshgrid(np.arange(64) + 64, np.arange(64) + 64, indexing="ij")
    return Workload("lowlou_n3_192x192_64x64x64_" + mapping, [Boundary(B0, x0, x0, h)], xyz,
                    np.array([0, xyz.shape[1]], np.int64), lam, fp32=False,
                    meta=dict(ll=ll, bottom_idx=(jj.ravel(), ii.ravel()), region_xy=rs))


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
