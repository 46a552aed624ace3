"""Pins of the oracle's gradient-consistency diagnostic (Sec. IV-B, Fig. 2):
the subset gradient against finite differences of the subset objective and of
the full objective, the subset gradients summing to the full one, the angle's
special cases, the smooth / variable areas on images whose gradient magnitude
is known in closed form, and the cyclic indexing of the angle sequence."""
import math

import numpy as np
import pytest

from tests.test_oracle_method import g2, g3, base_params


def data(orc, g, seed=0):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.5, 2.0, orc.n_voxels(g))
    q = orc.forward(g, f).reshape(-1)
    y = rng.poisson(q + 1.0).astype(float)
    r = np.full(y.size, 1.0)
    return f, y, r


@pytest.mark.parametrize("dim", [2, 3])
def test_subset_gradient_finite_differences(orc, dim):
    from oracle import gradcons as gc
    g = g2(orc) if dim == 2 else g3(orc)
    f, y, r = data(orc, g)
    beta, gR, eps = 0.3, 2.0, 1e-12
    rng = np.random.default_rng(1)
    d = rng.standard_normal(f.size)
    h = 1e-6
    for subset in (0, 1, g.n_subsets):
        gr = gc.subset_gradient(orc_g := g, f, y, r, subset, beta, gR, eps).reshape(-1)
        fd = (gc.subset_objective(orc_g, f + h * d, y, r, subset, beta, gR, eps)
              - gc.subset_objective(orc_g, f - h * d, y, r, subset, beta, gR, eps)) / (2 * h)
        assert abs(fd - gr @ d) <= 1e-6 * max(1.0, abs(fd)), (subset, fd, gr @ d)
    # subset 0 is Phi itself: the oracle's full objective
    full = gc.subset_gradient(g, f, y, r, 0, beta, gR, eps).reshape(-1)
    fd = (orc.objective(g, f + h * d, y, r, beta, gR, eps) - orc.objective(g, f - h * d, y, r, beta, gR, eps)) / (2 * h)
    assert abs(fd - full @ d) <= 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("dim", [2, 3])
def test_subset_gradients_sum_to_full(orc, dim):
    from oracle import gradcons as gc
    g = g2(orc) if dim == 2 else g3(orc)
    f, y, r = data(orc, g, 2)
    parts = sum(gc.subset_gradient(g, f, y, r, i, 0.5, 2.0, 1e-12) for i in range(1, g.n_subsets + 1))
    full = gc.subset_gradient(g, f, y, r, 0, 0.5, 2.0, 1e-12)
    assert np.max(np.abs(parts - full)) <= 1e-10 * np.max(np.abs(full))
    # and the subset objectives sum to Phi
    phis = sum(gc.subset_objective(g, f, y, r, i, 0.5, 2.0, 1e-12) for i in range(1, g.n_subsets + 1))
    assert phis == pytest.approx(orc.objective(g, f, y, r, 0.5, 2.0, 1e-12), rel=1e-12)


def test_angle_special_cases():
    from oracle.gradcons import angle
    v = np.array([1.0, -2.0, 3.0])
    assert angle(v, v) == pytest.approx(0.0, abs=1e-7)
    assert angle(v, 2.5 * v) == pytest.approx(0.0, abs=1e-7)
    assert angle(v, -v) == pytest.approx(math.pi)
    assert angle([1.0, 0.0], [0.0, 3.0]) == pytest.approx(math.pi / 2)
    assert angle([1.0, 0.0], [1.0, 1.0]) == pytest.approx(math.pi / 4)
    assert math.isnan(angle([], []))
    assert math.isnan(angle([0.0, 0.0], [1.0, 2.0]))


def test_areas_closed_forms(orc):
    """A plane f = a + c x + d y has gradient magnitude sqrt(c^2 + d^2) at
    every pixel (central and one-sided differences agree on it); a step
    between two levels has magnitude (jump / 2) on the two columns beside it
    and zero elsewhere."""
    from oracle import gradcons as gc
    g = g2(orc, n=8)
    yy, xx = np.mgrid[0:8, 0:8].astype(float)
    for c, d, smooth in ((1e-3, 2e-3, True), (0.3, 0.4, False)):
        f = 5.0 + c * xx + d * yy
        mean = 5.0 + 3.5 * (c + d)
        s, v = gc.areas(g, f)
        assert bool(s.all()) == smooth and bool(s.any()) == smooth
        assert v.all() == (math.hypot(c, d) > 0.2 * mean)
    f = np.where(xx < 4, 1.0, 2.0)      # mean 1.5: edge columns 3, 4 have 0.5 > 0.3
    s, v = gc.areas(g, f)
    assert np.array_equal(v, (xx == 3) | (xx == 4))
    assert np.array_equal(s, ~((xx == 3) | (xx == 4)))
    # 3D: the z slope counts
    g = g3(orc)
    zz = np.arange(g.nz, dtype=float)[:, None, None] * np.ones((1, g.ny, g.nx))
    f = 1.0 + 0.5 * zz
    s, v = gc.areas(g, f)
    assert v.all() and not s.any()


def test_sequence_indexing_with_frozen_iterate(orc):
    """With lambda_0 = 0 no subiteration moves f, so theta_{k,i} is the angle
    between grad Phi_{i-1} and grad Phi_i at f^0, with Phi_0 = Phi_M: for one
    subset every angle is zero, for two subsets theta_{k,1} = theta_{k,2},
    and every iteration repeats the first."""
    from oracle import gradcons as gc
    for M, check in ((1, "zero"), (2, "pair"), (3, "cycle")):
        g = g2(orc, M=M, na=12)
        f, y, r = data(orc, g, 4)
        f = 1.0 + 1e-4 * f          # smooth everywhere: I_s is the whole image
        p = base_params(orc, lambda0=0.0, beta=0.2)
        rec = orc.Recon(g, p, f.copy(), y, r)
        th, tt = gc.consistency_sequence(rec, 2)
        assert np.allclose(rec.f, f)
        assert th[0] == pytest.approx(th[1], abs=1e-12, nan_ok=True)
        if check == "zero":
            assert th[0][0] == pytest.approx(0.0, abs=1e-6)
        elif check == "pair":
            assert th[0][0] == pytest.approx(th[0][1], rel=1e-12)
            assert th[0][0] > 1e-3
        else:
            assert len(set(np.round(th[0], 12))) == 3
