"""The benchmark workloads (synthetic stand-ins for the paper's phantoms) and
the algorithm parameter defaults taken from the paper's tables.

Parameters (Sec. IV-A and Table II = tab:AlgorithmParameter_2D; Table III =
tab:AlgorithmParameter_3D): t = 1e-4, eps = 1e-12, gamma_R = 2, lambda0 = 1,
J0 = 3, J1 = 1000 (the printed "J_2" read as J1), delta2 = delta1 in 2D.
Subset counts outside Table II use the SDP-P2(12) row for M <= 12 and the
SDP-P2(24) row above; counts >= 1e6 use the high-count row and beta = 0.1,
else the low-count row and beta = 0.8.  3D uses the SDP-P2 non-TOF row of
Table III with beta = 0.1.
"""
from __future__ import annotations

import math

import numpy as np

from . import phantoms

DET_RADIUS_MM = 576 * 4.0 / (2 * math.pi)   # GE D710 ring: 576 detectors of 4 mm


def params_2d(M: int, counts: float, mode: str = "P2", U: float = 1e6) -> dict:
    high = counts >= 1e6
    base = dict(mode=mode, gamma_R=2.0, eps=1e-12, t_clip=1e-4, U=U, lambda0=1.0,
                J0=3, J1=1000, beta=0.1 if high else 0.8)
    if M <= 12:
        row = dict(a=1 / 5, rho=5.0, delta1=5.0, nu1=0.8, nu2=2.2) if high else \
            dict(a=1.3, rho=7.5, delta1=5.0, nu1=1.3, nu2=2.1)
        bsrem_a = (1 / 400) if high else (1 / 18)
        p1 = dict(a=1 / 13, nu1=1.6, nu2=2.4) if high else dict(a=0.5, nu1=1.6, nu2=2.4)
        m1_a, m2 = 1 / 50, dict(a=1 / 15, rho=3.0, delta1=1.0)
    else:
        row = dict(a=0.45, rho=4.0, delta1=3.0, nu1=0.8, nu2=1.8) if high else \
            dict(a=1.4, rho=2.2, delta1=1.0, nu1=1.3, nu2=2.4)
        bsrem_a = (1 / 35) if high else (1 / 5)
        p1 = dict(a=0.35, nu1=1.6, nu2=2.4) if high else dict(a=1.3, nu1=1.4, nu2=2.5)
        m1_a, m2 = 1 / 6, dict(a=1 / 5, rho=2.6, delta1=0.5)
    p = dict(base)
    p.update(row)
    if mode == "BSREM":
        p.update(a=bsrem_a)
    elif mode == "P1":
        p.update(p1)
    elif mode == "M1":
        p.update(a=m1_a)
    elif mode == "M2":
        p.update(m2)
    p["delta2"] = p["delta1"]
    return p


def params_2d_uniform(mode: str, U: float = 1e6) -> dict:
    """Table II, uniform phantom column (24 subsets, high count): BSREM, P1
    and P2; beta = 0.1 (high count).  Other modes take the brain-phantom
    rows (params_2d)."""
    p = params_2d(24, 1e7, mode=mode, U=U)
    if mode == "BSREM":
        p.update(a=1 / 35)
    elif mode == "P1":
        p.update(a=0.5, nu1=1.8, nu2=2.5)
    elif mode == "P2":
        p.update(a=0.7, rho=3.0, delta1=7.0, delta2=7.0, nu1=1.4, nu2=2.3)
    return p


# Sec. IV-A: total counts and the scatter / random fractions of the simulations
TC_HIGH, TC_LOW, SF, RF = 6.8e6, 6.8e5, 0.25, 0.25


def params_3d(U: float = 1e6, mode: str = "P2") -> dict:
    return dict(mode=mode, gamma_R=2.0, eps=1e-12, t_clip=1e-4, U=U, lambda0=1.6, a=1 / 4,
                rho=2.2, delta1=0.1, delta2=1.6, nu1=0.6, nu2=1.25, J0=0, J1=1000, beta=0.1)


def desc_2d(n, n_angles, n_radial, vx, M):
    return dict(dim=2, nx=n, ny=n, nz=1, vx=vx, vy=vx, vz=1.0, n_angles=n_angles,
                n_radial=n_radial, ds=vx, n_rings=1, max_ring_diff=0, ring_pitch=1.0,
                det_radius=DET_RADIUS_MM, n_subsets=M)


def desc_3d(n, nz, n_angles, n_radial, vx, vz, rings, max_rd, M):
    return dict(dim=3, nx=n, ny=n, nz=nz, vx=vx, vy=vx, vz=vz, n_angles=n_angles,
                n_radial=n_radial, ds=vx, n_rings=rings, max_ring_diff=max_rd, ring_pitch=vz,
                det_radius=DET_RADIUS_MM, n_subsets=M)


def c1():
    """2D, 64^2 (2 mm), 60 x 95, 4 subsets, 6 ellipses, 1e5 counts, 10 % background."""
    d = desc_2d(64, 60, 95, 2.0, 4)
    w = phantoms.make_2d(d, seed=11, n_ell=6, counts=1e5, bg_frac=0.1)
    return w, params_2d(4, 1e5, U=w.U), 10


def c2():
    """2D, 256^2 (300 mm FOV), 288 x 367, 24 subsets, 12 ellipses + 4 hot lesions,
    5e6 counts, 20 % background."""
    d = desc_2d(256, 288, 367, 300.0 / 256, 24)
    w = phantoms.make_2d(d, seed=12, n_ell=12, counts=5e6, bg_frac=0.2, hot_lesions=4)
    return w, params_2d(24, 5e6, U=w.U), 50


# Sec. IV-A: 32 parallel sub-rays per detector pair, Gaussian PSF of FWHM
# 6.59 mm, uniform water attenuation 0.096 / cm over the object's support
N_SUBRAYS, PSF_FWHM_MM, MU_WATER_PER_MM = 32, 6.59, 0.0096


def c2_full():
    """C2 with the paper's full 2D system model: 32 sub-rays per bin, the PSF,
    and attenuation by water over the phantom's support (the factors are
    computed from ``mu`` by the geometry, pet_os_attenuation_factors)."""
    w, p, n_iter = c2()
    w.desc = dict(w.desc, n_subrays=N_SUBRAYS, psf_fwhm=PSF_FWHM_MM)
    w.mu = np.where(w.f_true > 0, MU_WATER_PER_MM, 0.0)
    return w, p, n_iter


def c3(n=200, nz=64, n_angles=224, n_radial=281, max_rd=15, M=28, counts=5e8, seed=13):
    """Fully 3D: 200x200x64 (1.5 x 1.5 x 3 mm), 224 x 281, 64 rings, |d| <= 15, 28 subsets."""
    d = desc_3d(n, nz, n_angles, n_radial, 300.0 / n, 3.0, nz, max_rd, M)
    w = phantoms.make_3d(d, seed=seed, n_ell=11, counts=counts, bg_uniform=0.15, bg_scatter=0.15)
    return w, params_3d(U=w.U), 5


def c4_specs(n_recons=96, seed=14):
    """Shapes of the batched workload: n in {64..320 step 16}, M in 4..32,
    Na in [60, 360] rounded down to a multiple of M (>= 2M), Nr = 2 ceil(n/sqrt2) + 3."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_recons):
        n = int(rng.choice(np.arange(64, 321, 16)))
        M = int(rng.integers(4, 33))
        Na = int(rng.integers(60, 361))
        Na = max(2 * M, (Na // M) * M)
        Nr = 2 * int(math.ceil(n / math.sqrt(2))) + 3
        counts = float(10 ** rng.uniform(5, 7))
        n_ell = int(rng.integers(6, 13))
        out.append(dict(desc=desc_2d(n, Na, Nr, 300.0 / n, M), counts=counts, n_ell=n_ell,
                        seed=14000 + r, n_iter=10))
    return out


def c4_workload(spec):
    w = phantoms.make_2d(spec["desc"], seed=spec["seed"], n_ell=spec["n_ell"],
                         counts=spec["counts"], bg_frac=0.1)
    return w, params_2d(spec["desc"]["n_subsets"], spec["counts"], U=w.U), spec["n_iter"]


def c5_trace(n_requests=2000, rate=200.0, seed=15):
    """Poisson arrivals: 98 % 2D (n in 128..320 step 16, Na = 1.125 n rounded to a
    multiple of M, M in {8,12,16,24}), 2 % 3D (128x128x32, 180 x 185, 32 rings,
    |d| <= 7, M = 20); 30 iterations each."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < 0.02:
            desc = desc_3d(128, 32, 180, 185, 300.0 / 128, 300.0 / 128, 32, 7, 20)
            counts = 5e7
        else:
            n = int(rng.choice(np.arange(128, 321, 16)))
            M = int(rng.choice([8, 12, 16, 24]))
            Na = max(2 * M, int(round(1.125 * n / M)) * M)
            Nr = 2 * int(math.ceil(n / math.sqrt(2))) + 3
            desc = desc_2d(n, Na, Nr, 300.0 / n, M)
            counts = float(10 ** rng.uniform(5, 7))
        out.append(dict(arrival_s=t, desc=desc, counts=counts, seed=15000 + r, n_iter=30))
    return out
