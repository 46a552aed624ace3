"""Pins of the oracle's system matrix A (Siddon ray tracer) against things
other than itself: brute-force slab clipping, closed-form chords, the
theta = 0 column sum, 3D direct planes vs 2D, exact 90-degree symmetry,
analytic ellipse line integrals, and the adjoint identity.

A is the paper's ray-driven model (Sec. IV-A) with one line per bin."""
import math

import numpy as np
import pytest

from synth import phantoms


def g2(orc, n=6, na=12, nr=13, v=2.0, ds=None, M=3, nx=None):
    return orc.geom(dict(dim=2, nx=nx or n, ny=n, vx=v, vy=v, n_angles=na, n_radial=nr,
                         ds=ds if ds is not None else v, n_subsets=M))


def g3(orc, n=6, nz=4, na=8, nr=11, v=2.0, vz=3.0, D=2, M=2, Rd=60.0):
    return orc.geom(dict(dim=3, nx=n, ny=n, nz=nz, vx=v, vy=v, vz=vz, n_angles=na,
                         n_radial=nr, ds=v, n_rings=nz, max_ring_diff=D, ring_pitch=vz,
                         det_radius=Rd, n_subsets=M))


def dense_siddon(orc, g):
    P, nv = orc.n_planes(g), orc.n_voxels(g)
    A = np.zeros((P, g.n_angles, g.n_radial, nv))
    for p in range(P):
        for a in range(g.n_angles):
            for b in range(g.n_radial):
                vox, ln = orc.trace(g, p, a, b)
                np.add.at(A[p, a, b], vox, ln)
    return A.reshape(-1, nv)


def dense_clip(orc, g):
    P, nv = orc.n_planes(g), orc.n_voxels(g)
    nz = g.nz if g.dim == 3 else 1
    A = np.zeros((P, g.n_angles, g.n_radial, nv))
    for p in range(P):
        for a in range(g.n_angles):
            for b in range(g.n_radial):
                for iz in range(nz):
                    for iy in range(g.ny):
                        for ix in range(g.nx):
                            A[p, a, b, (iz * g.ny + iy) * g.nx + ix] = orc.chord_clip(g, p, a, b, ix, iy, iz)
    return A.reshape(-1, nv)


@pytest.mark.parametrize("n,na,nr,ds", [(6, 12, 13, 2.0),   # odd Nr, even n: axis rays on edges
                                        (6, 12, 12, 2.0),   # even Nr: axis rays through centres
                                        (5, 10, 11, 2.0),   # odd n
                                        (6, 9, 13, 1.5)])   # ds != v, odd Na (no pi/2)
def test_siddon_equals_bruteforce_clip_2d(orc, n, na, nr, ds):
    g = g2(orc, n=n, na=na, nr=nr, ds=ds)
    As, Ac = dense_siddon(orc, g), dense_clip(orc, g)
    assert np.abs(As - Ac).max() <= 1e-12 * Ac.max()
    assert (Ac > 0).sum() > 0


def test_siddon_equals_bruteforce_clip_3d(orc):
    g = g3(orc)
    As, Ac = dense_siddon(orc, g), dense_clip(orc, g)
    assert np.abs(As - Ac).max() <= 1e-12 * Ac.max()


def test_row_sum_is_chord_through_image_square(orc):
    """A 1 = length of the line inside the image rectangle (closed form)."""
    g = g2(orc, n=16, na=30, nr=25, v=1.5)
    q = orc.forward(g, np.ones((16, 16)))[0]
    c, s = phantoms.angle_table(30)
    sb = phantoms.bin_positions(25, 1.5)
    H = 8 * 1.5
    for a in range(30):
        for b in range(25):
            # parametric clip of x = sb c - u s, y = sb s + u c against [-H, H]^2
            lo, hi = -np.inf, np.inf
            inside = True
            for p0, d in ((sb[b] * c[a], -s[a]), (sb[b] * s[a], c[a])):
                if d == 0.0:
                    inside &= (-H <= p0 < H)
                    continue
                u0, u1 = sorted(((-H - p0) / d, (H - p0) / d))
                lo, hi = max(lo, u0), min(hi, u1)
            L = max(0.0, hi - lo) if inside else 0.0
            assert abs(q[a, b] - L) <= 1e-12 * 2 * H * 1.5


def test_single_pixel_chord_trapezoid(orc):
    """One-pixel image: q = chord through a square.  Closed form: the Radon
    transform of a box is the overlap of two intervals over |cos sin|."""
    n, v = 7, 2.0
    g = g2(orc, n=n, na=20, nr=31, v=v, ds=0.7)
    c, s = phantoms.angle_table(20)
    sb = phantoms.bin_positions(31, 0.7)
    for (ix, iy) in [(3, 3), (0, 6), (5, 1)]:
        f = np.zeros((n, n)); f[iy, ix] = 1.0
        q = orc.forward(g, f)[0]
        cx, cy = (ix - 3) * v, (iy - 3) * v
        for a in range(20):
            if c[a] == 0 or s[a] == 0:
                continue
            ha, hb = 0.5 * v * abs(c[a]), 0.5 * v * abs(s[a])
            u = sb - (cx * c[a] + cy * s[a])
            ov = np.clip(np.minimum(ha, u + hb) - np.maximum(-ha, u - hb), 0, None)
            ref = ov / abs(c[a] * s[a])
            assert np.allclose(q[a], ref, rtol=0, atol=1e-12 * v * 2)


def test_theta0_is_column_sum(orc):
    n, v = 10, 1.25
    g = g2(orc, n=n, na=6, nr=21, v=v)          # odd Nr, even n: rays on column edges
    rng = np.random.default_rng(0)
    f = rng.uniform(0, 1, (n, n))
    q = orc.forward(g, f)[0, 0]
    for b in range(21):
        col = (2 * b - 20 + n) // 2          # lower-edge convention: ray belongs to cell on its right
        ref = f[:, col].sum() * v if 0 <= col < n else 0.0
        assert abs(q[b] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_3d_direct_planes_equal_2d_slices(orc):
    g = g3(orc, n=8, nz=5, na=10, nr=13, D=2)
    g2d = g2(orc, n=8, na=10, nr=13, v=2.0, M=2)
    rng = np.random.default_rng(1)
    f = rng.uniform(0, 1, (5, 8, 8))
    q3 = orc.forward(g, f)
    for r in range(5):          # planes 0..R-1 are the direct planes d = 0
        assert orc.plane_rings(g, r) == (r, r)
        q2 = orc.forward(g2d, f[r])[0]
        assert np.abs(q3[r] - q2).max() <= 1e-12 * q2.max()


def test_rotation_by_90_degrees(orc):
    n = 12
    g = g2(orc, n=n, na=16, nr=19, v=1.0)
    rng = np.random.default_rng(2)
    f = rng.uniform(0, 1, (n, n))
    fr = np.empty_like(f)
    for iy in range(n):
        for ix in range(n):
            fr[iy, ix] = f[n - 1 - ix, iy]       # f'(x, y) = f(y, -x)
    q, qr = orc.forward(g, f)[0], orc.forward(g, fr)[0]
    for a in range(8):
        assert np.abs(qr[a + 8] - q[a]).max() <= 1e-12 * q.max()


def test_analytic_ellipse_convergence(orc):
    """Siddon projections of the rasterised phantom approach the exact line
    integrals of the ellipses at first order or better as pixels shrink."""
    rng = np.random.default_rng(3)
    ells = phantoms.random_ellipses(rng, 5, 60.0)
    na, nr, ds = 24, 61, 2.0
    exact = phantoms.analytic_sino_2d(ells, na, nr, ds)
    errs = []
    for n in (32, 64, 128):
        v = 120.0 / n
        g = orc.geom(dict(dim=2, nx=n, ny=n, vx=v, vy=v, n_angles=na, n_radial=nr, ds=ds, n_subsets=1))
        img = phantoms.raster_2d(ells, n, n, v, v, sub=8)
        q = orc.forward(g, img)[0]
        errs.append(np.linalg.norm(q - exact) / np.linalg.norm(exact))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.02
    assert min(orders) >= 0.8, (errs, orders)


def test_analytic_ellipsoid_3d(orc):
    """3D: every LOR of the rasterised ellipsoids approaches the exact line
    integral as voxels shrink (rings follow the slices, so each level is
    compared with the exact integrals along its own LORs)."""
    ells = [phantoms.Ellipse(3.0, -2.0, 14.0, 9.0, 0.4, 1.0, z0=1.0, C=7.0),
            phantoms.Ellipse(-5.0, 4.0, 6.0, 8.0, 1.1, 2.0, z0=-2.0, C=4.0)]
    errs = []
    for n, nz in ((16, 8), (32, 16), (64, 32)):
        v, vz = 40.0 / n, 24.0 / nz
        desc = dict(dim=3, nx=n, ny=n, nz=nz, vx=v, vy=v, vz=vz, n_angles=6, n_radial=17,
                    ds=2.5, n_rings=nz, max_ring_diff=2, ring_pitch=vz, det_radius=60.0, n_subsets=1)
        g = orc.geom(desc)
        img = phantoms.raster_3d(ells, n, n, nz, v, v, vz, sub=4)
        q = orc.forward(g, img)
        exact = phantoms.analytic_sino_3d(ells, 6, 17, 2.5, nz, 2, vz, 60.0)
        errs.append(np.linalg.norm(q - exact) / np.linalg.norm(exact))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.1 and min(orders) >= 0.7, (errs, orders)


@pytest.mark.parametrize("dim", [2, 3])
def test_adjoint_identity(orc, dim):
    g = g2(orc, n=20, na=18, nr=29, v=1.0, M=3) if dim == 2 else g3(orc, n=10, nz=6, na=8, nr=15, D=3, M=2)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, orc.n_voxels(g))
    y = rng.normal(0, 1, orc.n_bins(g))
    for subset in [0] + list(range(1, g.n_subsets + 1)):
        Ax = orc.forward(g, x, subset).reshape(-1)
        mask = np.zeros(orc.sino_shape(g), bool)
        for a in range(g.n_angles):
            if subset == 0 or a % g.n_subsets == subset - 1:
                mask[:, a, :] = True
        ym = np.where(mask.reshape(-1), y, 0.0)
        lhs = np.dot(Ax * mask.reshape(-1), ym)
        rhs = np.dot(x, orc.back(g, ym, subset).reshape(-1))
        assert abs(lhs - rhs) <= 1e-12 * (np.abs(Ax).dot(np.abs(ym)))


def test_subsets_partition_rows(orc):
    """Interleaved-angle subsets are disjoint and cover every row (Sec. II-B)."""
    g = g2(orc, n=8, na=12, nr=11, M=4)
    f = np.random.default_rng(6).uniform(0, 1, (8, 8))
    full = orc.forward(g, f, 0)
    acc = np.zeros_like(full)
    for i in range(1, 5):
        qi = orc.forward(g, f, i)
        for a in range(12):
            if a % 4 == i - 1:
                acc[:, a] += qi[:, a]
            else:
                assert not qi[:, a].any()
    assert np.array_equal(acc, full)


def test_sensitivity_and_pnorm(orc):
    g = g2(orc, n=8, na=2, nr=5, v=2.0, M=2)    # 0 and 90 degrees, 5 bins: corners unseen
    s = orc.sensitivity(g)
    assert np.isclose(s.sum(), orc.forward(g, np.ones((8, 8))).sum(), rtol=1e-13)
    p = orc.precond_norm(g, s)
    assert (s == 0).any()
    assert np.all(p[s == 0] == 1.0 / 2)
    assert np.allclose(p[s > 0], s[s > 0] / 2, rtol=1e-15)
