"""Host-side pieces of the convergence comparison (Sec. IV-A): the uniform
phantom, the SF/RF data model and the figures of merit."""
import numpy as np
import pytest

from synth import configs, phantoms
from paper_2111_07886_amd.convergence import iterations_to_reach, nrmsd


def test_uniform_phantom_geometry():
    img, rois = phantoms.uniform_phantom_2d(256)
    c = 127.5
    # background level 1, hot discs 10, cold discs 0 (area-weighted at edges)
    assert img[int(c), int(c)] == pytest.approx(1.0)
    for (rad, kind) in phantoms.UNIFORM_DISCS:
        m = rois[f"{kind}{rad}"]
        assert m.sum() > 0
        vals = img[m]
        assert np.allclose(vals, 10.0 if kind == "hot" else 0.0)
        # eroded ROI: pixel count close to pi (r-1)^2
        assert abs(m.sum() - np.pi * (rad - 1) ** 2) < 2 * np.pi * rad
    # the six discs do not overlap and lie inside the body
    assert img.max() == pytest.approx(10.0)
    total = img.sum()
    body = np.pi * 110.0 ** 2
    disc_extra = sum((9.0 if k == "hot" else -1.0) * np.pi * r ** 2 for r, k in phantoms.UNIFORM_DISCS)
    assert total == pytest.approx(body + disc_extra, rel=2e-3)
    assert rois["all"].sum() == sum(v.sum() for k, v in rois.items() if k != "all")


def test_sdp_data_model_fractions():
    rng = np.random.default_rng(3)
    Af = np.zeros((1, 60, 95))
    Af[0, :, 30:65] = rng.uniform(0.5, 2.0, size=(60, 35))
    TC = 6.8e6
    y, r, scale = phantoms.simulate_sdp_counts(Af, TC, rng, SF=configs.SF, RF=configs.RF)
    T = Af * scale
    R = np.full_like(T, configs.RF * TC / T.size)
    S = r - R
    assert T.sum() + S.sum() + R.sum() == pytest.approx(TC, rel=1e-12)
    assert S.sum() / (T.sum() + S.sum()) == pytest.approx(configs.SF, rel=1e-12)
    assert R.sum() / TC == pytest.approx(configs.RF, rel=1e-12)
    assert (S >= 0).all()
    # Poisson draw: total within 5 sigma of TC
    assert abs(y.sum() - TC) < 5 * np.sqrt(TC)
    assert np.array_equal(y, np.round(y))


def test_nrmsd_definition():
    g = np.array([[1.0, 2.0], [3.0, 4.0]])
    f = g + np.array([[0.0, 1.0], [0.0, -1.0]])
    assert nrmsd(f, g) == pytest.approx(np.sqrt(2.0 / 30.0))
    m = np.array([[False, True], [False, False]])
    assert nrmsd(f, g, m) == pytest.approx(0.5)
    assert nrmsd(g, g) == 0.0


def test_iterations_to_reach():
    phi = [10.0, 7.0, 5.0, 4.0, 3.5]
    assert iterations_to_reach(phi, 5.0) == 3
    assert iterations_to_reach(phi, 10.0) == 1
    assert iterations_to_reach(phi, 1.0) is None
