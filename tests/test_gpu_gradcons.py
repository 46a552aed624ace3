"""GPU parity of the gradient-consistency diagnostic (Sec. IV-B, Fig. 2)
through the C ABI against the FP64 oracle on the same FP32 inputs.

- subset gradient grad Phi_i(f): every term a_ij (1 - y_i/(A_i f + r_i)) is
  formed in FP32 (relative error a few 1e-7 each), so the error is bounded
  by a small multiple of 1e-7 * A_i^T (1 + y_i/(A_i f + r_i)) + the same
  relative size of the penalty term; the test allows 1e-5 of the norm of
  that magnitude bound (the same 1e-5 as the projectors);
- areas and angles on identical FP32 inputs: the area decisions are FP64 on
  both sides, so the sizes of I_s and I_v must be equal and the angles agree
  to 1e-9 rad (only the summation order differs).
"""
import math

import numpy as np
import pytest

from tests.test_gpu_parity import GEOMS, dev, f32, full_desc, host, rel, say, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = ["c1", "ragged_aniso", "3d_small", "3d_ragged"]


@pytest.fixture(scope="module")
def pet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_07886_amd as pet
    pet.lib()
    return pet


def iterate_after(orc, w, p, n_sub):
    rec = orc.Recon(orc.geom(w.desc), orc.params(p), w.f0, f32(w.y), f32(w.r))
    prev = None
    for _ in range(n_sub):
        prev = f32(rec.f)
        rec.subiteration()
    return f32(prev), f32(rec.f)


def magnitude_bound(orc, g, f, y, r, subset, p):
    from oracle import gradcons as gc
    q = orc.forward(g, f, subset)
    sel = gc._subset_rows(g, subset)
    m = np.zeros_like(q)
    ys, rs = y.reshape(q.shape), r.reshape(q.shape)
    m[sel] = 1.0 + ys[sel] / (q[sel] + rs[sel])
    wR = p["beta"] if subset == 0 else p["beta"] / g.n_subsets
    return orc.back(g, m, subset) + wR * np.abs(orc.rdp_grad(g, f, p["gamma_R"], p["eps"]))


@pytest.mark.parametrize("name", CASES + ["c2"])
def test_subset_gradient_parity(pet, orc, name):
    from oracle import gradcons as gc
    w, p, _ = workload(name, orc)
    M = w.desc["n_subsets"]
    g = orc.geom(w.desc)
    G = pet.Geometry(full_desc(w.desc))
    _, f = iterate_after(orc, w, p, M)          # the iterate after one oracle iteration
    f = f.reshape(G.img_shape)
    y, r = f32(w.y), f32(w.r)
    subsets = [0, 1, M] if name != "c2" else [0, 7]
    for subset in subsets:
        say(f"subset gradient {name} subset {subset}")
        hg = host(G.subset_gradient(p, dev(f), dev(y), dev(r), subset))
        ho = gc.subset_gradient(g, f, y, r, subset, p["beta"], p["gamma_R"], p["eps"])
        bound = magnitude_bound(orc, g, f, y, r, subset, p)
        e = float(np.linalg.norm(hg - ho) / np.linalg.norm(bound))
        say(f"  err / |bound| = {e:.2e}, rel-L2 = {rel(hg, ho):.2e}")
        assert e <= 1e-5, (subset, e)


@pytest.mark.parametrize("name", CASES + ["c2"])
def test_gradient_angles_parity(pet, orc, name):
    from oracle import gradcons as gc
    w, p, _ = workload(name, orc)
    M = w.desc["n_subsets"]
    g = orc.geom(w.desc)
    G = pet.Geometry(full_desc(w.desc))
    f_prev, f = iterate_after(orc, w, p, M + 1)
    f_prev, f = f_prev.reshape(G.img_shape), f.reshape(G.img_shape)
    y, r = f32(w.y), f32(w.r)
    hp = f32(gc.subset_gradient(g, f_prev, y, r, M, p["beta"], p["gamma_R"], p["eps"]))
    hc = f32(gc.subset_gradient(g, f, y, r, 1, p["beta"], p["gamma_R"], p["eps"]))
    nonempty = {"s": 0, "v": 0}
    for sf, vf in ((0.01, 0.2), (0.1, 0.05), (0.5, 0.01), (0.0, 1e9)):
        say(f"angles {name} thresholds {sf} {vf}")
        ts, tv, ns, nv = G.gradient_angles(dev(hp), dev(hc), dev(f), sf, vf)
        os_, ov, ons, onv = gc.gradient_angles(g, hp, hc, f, sf, vf)
        assert (ns, nv) == (ons, onv)
        for a, b in ((ts, os_), (tv, ov)):
            if math.isnan(b):
                assert math.isnan(a)
            else:
                assert abs(a - b) <= 1e-9, (a, b)
        nonempty["s"] += ns > 0
        nonempty["v"] += nv > 0
    assert nonempty["s"] >= 2 and nonempty["v"] >= 2


def test_angles_of_identical_and_opposite_vectors(pet, orc):
    """theta(h, h) = 0, theta(h, -h) = pi on every area, and an all-zero
    restriction gives NaN, on a 3D image (the z slope counts in grad f)."""
    d = full_desc(GEOMS["3d_ragged"])
    G = pet.Geometry(d)
    rng = np.random.default_rng(7)
    h = dev(rng.standard_normal(G.img_shape))
    zz = np.arange(d["nz"], dtype=float)[:, None, None] * np.ones((1, d["ny"], d["nx"]))
    f = dev(1.0 + 0.5 * zz)                # grad f = 0.5 everywhere (central and one-sided alike)
    ts, tv, ns, nv = G.gradient_angles(h, h, f, 0.01, 0.05)
    assert ns == 0 and nv == G.n_voxels and math.isnan(ts) and tv == pytest.approx(0.0, abs=1e-6)
    ts, tv, ns, nv = G.gradient_angles(h, -h, f, 0.01, 0.05)
    assert tv == pytest.approx(math.pi, abs=1e-6)
    ts, tv, ns, nv = G.gradient_angles(torch.zeros_like(h), h, f, 0.01, 0.05)
    assert math.isnan(tv)


def test_sequence_with_frozen_iterate(pet, orc):
    """lambda_0 tiny: f does not move, so with two subsets theta_{k,1} and
    theta_{k,2} are the same angle (bitwise: the FP64 sums are formed in a
    fixed order from the same products), and with one subset it is zero."""
    from paper_2111_07886_amd.diagnostics import gradient_consistency
    from synth import configs
    for M in (1, 2):
        d = full_desc(dict(GEOMS["c1"], n_subsets=M))
        G = pet.Geometry(d)
        w, _, _ = configs.c1()
        p = configs.params_2d(4, 1e5, mode="P2", U=w.U)
        p.update(lambda0=1e-30)
        rng = np.random.default_rng(3)
        f = dev(1.0 + 1e-4 * rng.uniform(size=G.img_shape))
        f0 = host(f)
        out = gradient_consistency(G, p, f, dev(w.y), dev(w.r), 2)
        assert np.array_equal(host(f), f0)
        th = out["theta"]
        assert th[0] == th[1]
        if M == 1:
            assert th[0][0] == pytest.approx(0.0, abs=1e-6)
        else:
            assert th[0][0] == th[0][1] and th[0][0] > 1e-3


def test_invalid_arguments(pet):
    d = full_desc(GEOMS["c1"])
    G = pet.Geometry(d)
    h = torch.zeros(G.img_shape, device="cuda")
    with pytest.raises(pet.PetOSError):
        G.gradient_angles(h, h, h, -1.0, 0.2)
    from synth import configs
    p = configs.params_2d(4, 1e5, U=10.0)
    y = torch.ones(G.sino_shape, device="cuda")
    with pytest.raises(pet.PetOSError):
        G.subset_gradient(p, h, y, y, d["n_subsets"] + 1)
