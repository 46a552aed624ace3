"""Pins of the oracle's full 2D system model of Sec. IV-A, A = diag(att) P B:
P the mean over n_sub parallel sub-rays per bin, B the Gaussian PSF (FWHM),
att per-bin attenuation factors.

- sub-ray traces against brute-force slab clipping of the same lines;
- row sums against the closed-form chord of each sub-ray through the image
  rectangle (a trapezoid in the line's offset);
- per-angle sensitivity of a pixel against its area / ds (sub-rays tile the
  detector with spacing ds / n_sub);
- the PSF is symmetric, keeps linear images, and its discrete variance is
  the Gaussian's sigma^2 = (FWHM / 2 sqrt(2 ln 2))^2 up to the 3-sigma cut;
- the attenuation factors multiply rows; the whole operator is the adjoint
  of the back-projection; the fidelity gradient matches finite differences.
"""
import math

import numpy as np
import pytest


def geo(orc, n=8, na=12, nr=13, v=2.0, M=3, ns=1, fwhm=0.0, att=None, ny=None):
    return orc.geom(dict(dim=2, nx=n, ny=ny or n, vx=v, vy=v, n_angles=na, n_radial=nr, ds=v, n_subsets=M,
                         n_subrays=ns, psf_fwhm=fwhm, att=att))


def dense(orc, g, ns):
    P = orc.n_planes(g)
    A = np.zeros((g.n_angles * g.n_radial, orc.n_voxels(g)))
    row = 0
    for a in range(g.n_angles):
        for b in range(g.n_radial):
            for iy in range(g.ny):
                for ix in range(g.nx):
                    s = 0.0
                    for k in range(ns):
                        s += orc.chord_clip_off(g, 0, a, b, orc.subray_offset(g, k), ix, iy, 0)
                    A[row, iy * g.nx + ix] = s / ns
            row += 1
    return A


@pytest.mark.parametrize("ns", [1, 4, 32])
def test_subray_trace_against_clipping(orc, ns):
    g = geo(orc, n=6, na=8, nr=9, ns=ns)
    A = dense(orc, g, ns)
    rng = np.random.default_rng(0)
    f = rng.uniform(0.0, 1.0, 36)
    q = orc.forward(g, f).reshape(-1)
    assert np.max(np.abs(q - A @ f)) <= 1e-12 * np.max(np.abs(q))
    w = rng.uniform(-1.0, 1.0, q.size)
    assert np.max(np.abs(orc.back(g, w).reshape(-1) - A.T @ w)) <= 1e-12 * np.max(np.abs(A.T @ w))


def rect_chord(W, H, c, s, t):
    """Length of the line x c + y s = t inside the centred W x H rectangle."""
    e_out = 0.5 * (W * abs(c) + H * abs(s))
    e_in = 0.5 * abs(W * abs(c) - H * abs(s))
    Lmax = min(W / abs(s) if s != 0 else math.inf, H / abs(c) if c != 0 else math.inf)
    at = abs(t)
    if at >= e_out:
        return 0.0
    if at <= e_in or e_out == e_in:
        return Lmax
    return Lmax * (e_out - at) / (e_out - e_in)


def test_row_sums_closed_form(orc):
    ns = 32
    g = geo(orc, n=10, ny=7, na=10, nr=17, v=1.5, ns=ns)
    W, H = 10 * 1.5, 7 * 1.5
    q = orc.forward(g, np.ones((7, 10)))
    for a in range(1, g.n_angles):
        if 2 * a == g.n_angles:
            continue          # axis-parallel: edge rule, checked by clipping
        c, s = orc.angle(g, a)
        for b in range(g.n_radial):
            sb = (b - 0.5 * (g.n_radial - 1)) * g.ds
            ref = sum(rect_chord(W, H, c, s, sb + orc.subray_offset(g, k)) for k in range(ns)) / ns
            assert q[0, a, b] == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_per_angle_sensitivity_is_pixel_area_over_ds(orc):
    """With 32 sub-rays per bin the sub-rays sample the detector every ds/32:
    a pixel well inside the field collects (sum of its chords)/32 ~ its area
    / ds per angle (to the sampling error of a trapezoid, < 1e-3)."""
    ns = 32
    g = geo(orc, n=9, na=7, nr=15, v=2.0, ns=ns)
    for a in range(g.n_angles):
        e = np.zeros(g.n_angles * g.n_radial)
        e.reshape(g.n_angles, g.n_radial)[a, :] = 1.0
        s = orc.back(g, e)
        assert s[4, 4] == pytest.approx(2.0 * 2.0 / g.ds, rel=1e-3)


def test_psf_symmetric_linear_and_variance(orc):
    fwhm = 6.59
    g = geo(orc, n=40, v=1.171875, fwhm=fwhm)
    K = orc.psf_radius(g, g.vx)
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal((40, 40)), rng.standard_normal((40, 40))
    assert np.sum(orc.blur(g, x) * y) == pytest.approx(np.sum(x * orc.blur(g, y)), rel=1e-12)
    yy, xx = np.mgrid[0:40, 0:40].astype(float)
    lin = 3.0 + 0.5 * xx - 0.25 * yy
    inner = (slice(K, 40 - K), slice(K, 40 - K))
    assert np.allclose(orc.blur(g, lin)[inner], lin[inner], rtol=0, atol=1e-12)
    # blur of x^2 (in mm) adds the kernel's variance along x
    X = (xx - 20) * g.vx
    var = (orc.blur(g, X * X) - X * X)[inner]
    sigma2 = (fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))) ** 2
    assert np.allclose(var, var.flat[0], rtol=1e-9)
    assert var.flat[0] == pytest.approx(sigma2, rel=0.03)
    assert var.flat[0] < sigma2
    # mass kept for an image away from the border
    f = np.zeros((40, 40))
    f[15:25, 12:20] = rng.uniform(size=(10, 8))
    assert orc.blur(g, f).sum() == pytest.approx(f.sum(), rel=1e-12)


def test_attenuation_rows_adjoint_and_gradient(orc):
    rng = np.random.default_rng(4)
    base = dict(n=8, na=12, nr=13, v=2.0, M=3, ns=4, fwhm=5.0)
    att = rng.uniform(0.3, 1.0, 12 * 13)
    g0 = geo(orc, **base)
    g = geo(orc, **base, att=att)
    f = rng.uniform(0.5, 2.0, 64)
    q0 = orc.forward(g0, f).reshape(-1)
    assert np.allclose(orc.forward(g, f).reshape(-1), att * q0, rtol=1e-14, atol=0)
    w = rng.uniform(-1.0, 1.0, q0.size)
    assert np.allclose(orc.back(g, w), orc.back(g0, att * w), rtol=1e-13, atol=1e-14)
    # adjoint pair of the whole operator, subset by subset
    for subset in (0, 2):
        qa = orc.forward(g, f, subset).reshape(-1)
        bw = orc.back(g, w, subset).reshape(-1)
        assert np.dot(qa, w) == pytest.approx(np.dot(f, bw), rel=1e-12)
    # fidelity gradient by finite differences
    y = rng.poisson(q0 * att + 1.0).astype(float)
    r = np.full(y.size, 1.0)
    q = orc.forward(g, f).reshape(-1)
    grad = orc.back(g, 1.0 - y / (q + r)).reshape(-1)
    # central differences: truncation O(h^2), rounding ~1e-16 |F| / h
    h = 1e-4
    d = rng.standard_normal(64)
    F = orc.fidelity(g, f, y, r)
    fd = (orc.fidelity(g, f + h * d, y, r) - orc.fidelity(g, f - h * d, y, r)) / (2 * h)
    assert abs(fd - grad @ d) <= 1e-6 * abs(grad @ d) + 1e-14 * abs(F) / h
