"""Seeded synthetic PET inputs shared by the oracle tests and the GPU path.

Holds none of the reconstruction's arithmetic: phantoms are rasterised
ellipses / ellipsoids, measured data are *analytic* line integrals of those
shapes (not the pixel system matrix), scaled to a count level, plus a
uniform (and optionally smoothed-projection "scatter") background, with
Poisson noise (model-Poisson in Sec. II-A; data simulation of Sec. IV-A).

The ray geometry used to evaluate the analytic line integrals follows the
shared conventions: pixel centres at (i - (n-1)/2) v, angles a*pi/Na with
(cos,sin) snapped at 0 and pi/2, bins (b - (Nr-1)/2) ds, line
x cos + y sin = s with direction (-sin, cos); in 3D the LOR rises linearly
from ring r1 at u = -h to ring r2 at u = +h, h = sqrt(Rd^2 - s^2), rings at
slice centres, span-1 plane order d = 0, +1, -1, ..., ascending r1.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# ray geometry (conventions only)
# ----------------------------------------------------------------------------

def angle_table(n_angles: int):
    a = np.arange(n_angles)
    th = a * math.pi / n_angles
    c, s = np.cos(th), np.sin(th)
    c[0], s[0] = 1.0, 0.0
    if n_angles % 2 == 0:
        c[n_angles // 2], s[n_angles // 2] = 0.0, 1.0
    return c, s


def bin_positions(n_radial: int, ds: float):
    return (np.arange(n_radial) - 0.5 * (n_radial - 1)) * ds


def plane_table(n_rings: int, max_ring_diff: int):
    """(r1, r2) per plane in span-1 order d = 0, +1, -1, +2, -2, ..."""
    out = []
    for m in range(2 * max_ring_diff + 1):
        d = 0 if m == 0 else ((m + 1) // 2 if m % 2 else -(m // 2))
        lo = -d if d < 0 else 0
        hi = n_rings - 1 if d < 0 else n_rings - 1 - d
        for r1 in range(lo, hi + 1):
            out.append((r1, r1 + d))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


# ----------------------------------------------------------------------------
# shapes
# ----------------------------------------------------------------------------

@dataclass
class Ellipse:
    x0: float
    y0: float
    A: float          # semi-axis along the rotated x'
    B: float
    phi: float        # rotation of x' from x
    val: float
    z0: float = 0.0   # 3D only
    C: float = 0.0    # 3D semi-axis along z (0 => 2D ellipse)


def random_ellipses(rng, n, r_img, val_lo=0.5, val_hi=4.0):
    out = []
    for _ in range(n):
        rad = r_img * 0.5 * math.sqrt(rng.uniform())
        ang = rng.uniform(0, 2 * math.pi)
        out.append(Ellipse(x0=rad * math.cos(ang), y0=rad * math.sin(ang),
                           A=rng.uniform(0.1, 0.45) * r_img, B=rng.uniform(0.1, 0.45) * r_img,
                           phi=rng.uniform(0, math.pi), val=rng.uniform(val_lo, val_hi)))
    return out


def raster_2d(ells, nx, ny, vx, vy, sub=4):
    """Mean of sub x sub point samples per pixel of the additive ellipse sum."""
    img = np.zeros((ny, nx))
    off = (np.arange(sub) + 0.5) / sub - 0.5
    xc = (np.arange(nx) - 0.5 * (nx - 1)) * vx
    yc = (np.arange(ny) - 0.5 * (ny - 1)) * vy
    for dy in off:
        for dx in off:
            X = (xc + dx * vx)[None, :]
            Y = (yc + dy * vy)[:, None]
            for e in ells:
                cp, sp = math.cos(e.phi), math.sin(e.phi)
                xr = (X - e.x0) * cp + (Y - e.y0) * sp
                yr = -(X - e.x0) * sp + (Y - e.y0) * cp
                img += e.val * ((xr / e.A) ** 2 + (yr / e.B) ** 2 <= 1.0)
    return img / (sub * sub)


def raster_3d(ells, nx, ny, nz, vx, vy, vz, sub=2):
    img = np.zeros((nz, ny, nx))
    off = (np.arange(sub) + 0.5) / sub - 0.5
    xc = (np.arange(nx) - 0.5 * (nx - 1)) * vx
    yc = (np.arange(ny) - 0.5 * (ny - 1)) * vy
    zc = (np.arange(nz) - 0.5 * (nz - 1)) * vz
    for dz in off:
        for dy in off:
            for dx in off:
                X = (xc + dx * vx)[None, None, :]
                Y = (yc + dy * vy)[None, :, None]
                Z = (zc + dz * vz)[:, None, None]
                for e in ells:
                    cp, sp = math.cos(e.phi), math.sin(e.phi)
                    xr = (X - e.x0) * cp + (Y - e.y0) * sp
                    yr = -(X - e.x0) * sp + (Y - e.y0) * cp
                    img += e.val * ((xr / e.A) ** 2 + (yr / e.B) ** 2 + ((Z - e.z0) / e.C) ** 2 <= 1.0)
    return img / sub ** 3


def analytic_sino_2d(ells, n_angles, n_radial, ds):
    """Exact line integrals [angle][bin] of the additive ellipse phantom."""
    c, s = angle_table(n_angles)
    sb = bin_positions(n_radial, ds)
    out = np.zeros((n_angles, n_radial))
    for e in ells:
        th_c = c * math.cos(e.phi) + s * math.sin(e.phi)        # cos(theta - phi)
        th_s = s * math.cos(e.phi) - c * math.sin(e.phi)        # sin(theta - phi)
        a2 = (e.A * th_c) ** 2 + (e.B * th_s) ** 2
        sp = sb[None, :] - (e.x0 * c + e.y0 * s)[:, None]
        disc = a2[:, None] - sp ** 2
        out += np.where(disc > 0, 2 * e.val * e.A * e.B * np.sqrt(np.maximum(disc, 0)) / a2[:, None], 0.0)
    return out


def analytic_sino_3d(ells, n_angles, n_radial, ds, n_rings, max_ring_diff, ring_pitch, det_radius,
                     planes_per_chunk=16):
    """Exact 3D line integrals [plane][angle][bin] of an additive ellipsoid phantom."""
    c, s = angle_table(n_angles)
    sb = bin_positions(n_radial, ds)
    pt = plane_table(n_rings, max_ring_diff)
    zr = (np.arange(n_rings) - 0.5 * (n_rings - 1)) * ring_pitch
    h = np.sqrt(det_radius ** 2 - sb ** 2)                         # [b]
    # transaxial point at u = 0 and direction, [a][b]
    px = (sb[None, :] * c[:, None]).reshape(-1)
    py = (sb[None, :] * s[:, None]).reshape(-1)
    dx = np.repeat(-s, n_radial)
    dy = np.repeat(c, n_radial)
    hb = np.tile(h, n_angles)
    out = np.zeros((len(pt), n_angles * n_radial), dtype=np.float64)

    def chunk(p0):
        sl = slice(p0, min(len(pt), p0 + planes_per_chunk))
        z1 = zr[pt[sl, 0]][:, None]
        z2 = zr[pt[sl, 1]][:, None]
        mz = (z2 - z1) / (2 * hb[None, :])                           # dz/du
        zc0 = z1 + mz * hb[None, :]                                  # z at u = 0
        kappa = np.sqrt(1 + mz ** 2)
        acc = np.zeros_like(mz)
        for e in ells:
            cp, sp = math.cos(e.phi), math.sin(e.phi)
            ex = (px - e.x0) * cp + (py - e.y0) * sp
            ey = -(px - e.x0) * sp + (py - e.y0) * cp
            qx = dx * cp + dy * sp
            qy = -dx * sp + dy * cp
            at = (qx / e.A) ** 2 + (qy / e.B) ** 2
            bt = ex * qx / e.A ** 2 + ey * qy / e.B ** 2
            ct = (ex / e.A) ** 2 + (ey / e.B) ** 2
            pz = zc0 - e.z0
            a = at[None, :] + (mz / e.C) ** 2
            b = bt[None, :] + pz * mz / e.C ** 2
            cc = ct[None, :] + (pz / e.C) ** 2 - 1.0
            disc = b * b - a * cc
            acc += np.where(disc > 0, e.val * 2.0 * np.sqrt(np.maximum(disc, 0)) / a, 0.0) * kappa
        out[sl] = acc

    # numpy releases the GIL inside these array expressions: chunks of planes
    # run on a thread pool
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(chunk, range(0, len(pt), planes_per_chunk)))
    return out.reshape(len(pt), n_angles, n_radial)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    desc: dict                  # geometry descriptor (C-ABI keys)
    f_true: np.ndarray          # scaled pixelised phantom (reference only)
    y: np.ndarray               # counts, natural layout [plane][angle][bin]
    r: np.ndarray               # background mean (> 0)
    f0: np.ndarray              # initial image (ones, Sec. IV-A)
    U: float                    # box bound used by both sides
    meta: dict = field(default_factory=dict)


def _smooth_bins(x, sigma_bins):
    """Gaussian blur along the radial-bin axis (zero outside the sinogram)."""
    from scipy.ndimage import gaussian_filter1d
    return gaussian_filter1d(x, sigma_bins, axis=-1, mode="constant", truncate=4.0)


def make_2d(desc, seed, n_ell, counts, bg_frac, hot_lesions=0, lesion_diam_px=5, lesion_contrast=4.0):
    rng = np.random.default_rng(seed)
    nx, ny, vx, vy = desc["nx"], desc["ny"], desc["vx"], desc["vy"]
    r_img = 0.5 * min(nx * vx, ny * vy)
    ells = random_ellipses(rng, n_ell, r_img)
    base = raster_2d(ells, nx, ny, vx, vy)
    lesions = []
    tries = 0
    while len(lesions) < hot_lesions and tries < 10000:
        tries += 1
        ix, iy = rng.integers(lesion_diam_px, nx - lesion_diam_px), rng.integers(lesion_diam_px, ny - lesion_diam_px)
        local = base[iy, ix]
        if local <= 0:
            continue
        x0 = (ix - 0.5 * (nx - 1)) * vx
        y0 = (iy - 0.5 * (ny - 1)) * vy
        rad = 0.5 * lesion_diam_px * vx
        lesions.append(Ellipse(x0=x0, y0=y0, A=rad, B=rad, phi=0.0, val=(lesion_contrast - 1.0) * local))
    ells = ells + lesions
    img = raster_2d(ells, nx, ny, vx, vy) if lesions else base
    sino = analytic_sino_2d(ells, desc["n_angles"], desc["n_radial"], desc["ds"])[None]
    scale = counts / sino.sum()
    trues = sino * scale
    gamma = np.full_like(trues, bg_frac * counts / trues.size)
    y = rng.poisson(trues + gamma).astype(np.float64)
    f_true = img * scale
    f0 = np.ones((ny, nx))
    U = 1e3 * max(1.0, float(f_true.max()))
    return Workload(desc=desc, f_true=f_true, y=y, r=gamma, f0=f0, U=U,
                    meta=dict(seed=seed, counts=counts, bg_frac=bg_frac, n_ellipses=n_ell,
                              hot_lesions=len(lesions)))


def make_3d(desc, seed, n_ell, counts, bg_uniform, bg_scatter, scatter_sigma_bins=20.0):
    rng = np.random.default_rng(seed)
    nx, ny, nz = desc["nx"], desc["ny"], desc["nz"]
    vx, vy, vz = desc["vx"], desc["vy"], desc["vz"]
    r_img = 0.5 * min(nx * vx, ny * vy)
    hz = 0.5 * nz * vz
    body = Ellipse(0.0, 0.0, 0.8 * r_img, 0.6 * r_img, 0.0, 1.0, z0=0.0, C=0.85 * hz)
    ells = [body]
    for e in random_ellipses(rng, n_ell, 0.7 * r_img):
        e.A *= 0.5
        e.B *= 0.5
        e.z0 = rng.uniform(-0.5, 0.5) * hz
        e.C = rng.uniform(0.15, 0.4) * hz
        ells.append(e)
    img = raster_3d(ells, nx, ny, nz, vx, vy, vz)
    sino = analytic_sino_3d(ells, desc["n_angles"], desc["n_radial"], desc["ds"], desc["n_rings"],
                            desc["max_ring_diff"], desc["ring_pitch"], desc["det_radius"])
    scale = counts / sino.sum()
    trues = sino * scale
    n = trues.size
    gamma = np.full_like(trues, bg_uniform * counts / n)
    if bg_scatter > 0:
        sc = _smooth_bins(trues, scatter_sigma_bins)
        gamma += sc * (bg_scatter * counts / sc.sum())
    y = rng.poisson(trues + gamma).astype(np.float64)
    f_true = img * scale
    f0 = np.ones((nz, ny, nx))
    U = 1e3 * max(1.0, float(f_true.max()))
    return Workload(desc=desc, f_true=f_true, y=y, r=gamma, f0=f0, U=U,
                    meta=dict(seed=seed, counts=counts, bg_uniform=bg_uniform, bg_scatter=bg_scatter,
                              n_ellipsoids=len(ells)))


# ----------------------------------------------------------------------------
# the uniform phantom and data model of the paper's simulations (Sec. IV-A)
# ----------------------------------------------------------------------------

UNIFORM_DISCS = ((4, "hot"), (6, "hot"), (8, "cold"), (10, "cold"), (12, "hot"), (14, "hot"))


def uniform_phantom_2d(n=256, body_radius_px=110.0, ring_radius_px=70.0, hot=10.0, sub=4):
    """Uniform phantom of Fig. 1b / Sec. IV-A: a uniform background disc with
    six discs of radii 4, 6, 8 (cold), 10 (cold), 12 and 14 pixels, contrast
    0:1 (cold) and 10:1 (hot, our reading of the printed "1:10").  The paper
    gives no positions: the discs sit on a ring of ring_radius_px around the
    centre, 60 degrees apart, inside a body of radius body_radius_px.  The
    image is rasterised with sub x sub supersampling (unit pixel pitch).

    ROIs (Fig. 6): each disc, a background disc of radius 25 px at the centre,
    and "all" = their union; an ROI takes the pixels whose centre lies at least
    one pixel inside its disc edge."""
    c = 0.5 * (n - 1)
    s = (np.arange(sub) + 0.5) / sub - 0.5
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    discs = []
    for k, (rad, kind) in enumerate(UNIFORM_DISCS):
        th = 2.0 * np.pi * k / 6.0
        discs.append((c + ring_radius_px * np.cos(th), c + ring_radius_px * np.sin(th), float(rad), kind))
    img = np.zeros((n, n))
    for dy in s:
        for dx in s:
            px, py = xx + dx, yy + dy
            v = ((px - c) ** 2 + (py - c) ** 2 <= body_radius_px ** 2).astype(np.float64)
            for cx, cy, rad, kind in discs:
                inside = (px - cx) ** 2 + (py - cy) ** 2 <= rad ** 2
                v = np.where(inside, hot if kind == "hot" else 0.0, v)
            img += v
    img /= sub * sub
    rois = {}
    for (cx, cy, rad, kind), (r0, _) in zip(discs, UNIFORM_DISCS):
        rois[f"{kind}{int(r0)}"] = (xx - cx) ** 2 + (yy - cy) ** 2 <= (rad - 1.0) ** 2
    rois["background"] = (xx - c) ** 2 + (yy - c) ** 2 <= 25.0 ** 2
    allm = np.zeros((n, n), bool)
    for m in rois.values():
        allm |= m
    rois["all"] = allm
    return img, rois


def simulate_sdp_counts(Af, TC, rng, SF=0.25, RF=0.25, scatter_sigma_bins=20.0):
    """Data model of Sec. IV-A without the PSF and the attenuation: trues are
    the projection Af of the phantom through the reconstruction system matrix,
    scatter a smoothed copy of it scaled to SF = S/(T+S), randoms uniform with
    RF = R/(T+S+R), total mean count TC = T+S+R; y is Poisson.  Returns
    (y, r, scale) with r = S + R the known background mean and scale the
    factor that turns the phantom into the activity whose projection is T."""
    Af = np.asarray(Af, dtype=np.float64)
    T_tot = (1.0 - SF) * (1.0 - RF) * TC
    S_tot = SF * (1.0 - RF) * TC
    R_tot = RF * TC
    scale = T_tot / Af.sum()
    T = Af * scale
    sm = _smooth_bins(Af, scatter_sigma_bins)
    S = sm * (S_tot / sm.sum())
    R = np.full_like(T, R_tot / T.size)
    r = S + R
    y = rng.poisson(T + r).astype(np.float64)
    return y, r, scale
