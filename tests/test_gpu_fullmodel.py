"""GPU parity of the full 2D system model of Sec. IV-A (A = diag(att) P B:
P the mean over parallel sub-rays per bin, B the Gaussian PSF, att per-bin
attenuation factors) through the C ABI, against the FP64 oracle on the same
FP32 inputs: sensitivity, projections, attenuation factors, the adjoint
identity, one subiteration from the oracle's own state (SDP-P2 and OSEM),
and the subset gradient.  Tolerances as for the single-line model (rel-L2
1e-5); the sub-ray weights are evaluated in FP32 from an FP64 offset."""
import math

import numpy as np
import pytest

from tests.test_gpu_parity import dev, f32, full_desc, host, rel, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MU_WATER = 0.0096    # 1/mm (0.096 / cm, Sec. IV-A)

BASE = {
    "c1": dict(dim=2, nx=64, ny=64, vx=2.0, vy=2.0, n_angles=60, n_radial=95, ds=2.0, n_subsets=4),
    "ragged": dict(dim=2, nx=50, ny=37, vx=2.0, vy=2.5, n_angles=30, n_radial=71, ds=1.7, n_subsets=5),
    "c2": dict(dim=2, nx=256, ny=256, vx=300 / 256, vy=300 / 256, n_angles=288, n_radial=367, ds=300 / 256,
               n_subsets=24),
}
MODELS = {
    "sub32": dict(n_subrays=32),
    "psf": dict(psf_fwhm=6.59),
    "full": dict(n_subrays=32, psf_fwhm=6.59, att=True),
    "full8": dict(n_subrays=8, psf_fwhm=5.0, att=True),
}
CASES = [("c1", "sub32"), ("c1", "psf"), ("c1", "full"), ("ragged", "full8"), ("c2", "full")]


@pytest.fixture(scope="module")
def pet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_07886_amd as pet
    pet.lib()
    return pet


def support_mu(d):
    """Uniform water over an elliptical body support (the object's support)."""
    yy, xx = np.mgrid[0:d["ny"], 0:d["nx"]].astype(float)
    X = (xx - 0.5 * (d["nx"] - 1)) * d["vx"]
    Y = (yy - 0.5 * (d["ny"] - 1)) * d["vy"]
    a, b = 0.42 * d["nx"] * d["vx"], 0.36 * d["ny"] * d["vy"]
    return np.where((X / a) ** 2 + (Y / b) ** 2 <= 1.0, MU_WATER, 0.0)


_cache = {}


def make(pet, orc, base, model):
    key = (base, model)
    if key in _cache:
        return _cache[key]
    m = dict(MODELS[model])
    use_att = m.pop("att", False)
    d = full_desc(dict(BASE[base], **m))
    att = None
    if use_att:
        G0 = pet.Geometry(dict(d, psf_fwhm=0.0))
        att = host(G0.attenuation_factors(dev(support_mu(d)))).astype(np.float32)
        G0.close()
    G = pet.Geometry(d, att=att)
    g = orc.geom(dict(d, att=None if att is None else att.astype(np.float64)))
    _cache[key] = (G, g, d, att)
    return _cache[key]


def data(orc, g, d, seed):
    rng = np.random.default_rng(seed)
    shape = (d["ny"], d["nx"])
    yy, xx = np.mgrid[0:d["ny"], 0:d["nx"]].astype(float)
    f_true = 1.0 + 3.0 * ((xx - d["nx"] / 2) ** 2 + (yy - d["ny"] / 3) ** 2 < (d["nx"] / 6) ** 2)
    f_true = f_true * (support_mu(d) > 0)
    q = orc.forward(g, f_true)
    r = np.full(q.shape, 0.2 * q.mean())
    y = rng.poisson(50.0 * (q + r) / q.mean()) * q.mean() / 50.0
    return f32(np.ones(shape)), f32(y), f32(r)


@pytest.mark.parametrize("base,model", CASES)
def test_sensitivity(pet, orc, base, model):
    G, g, _, _ = make(pet, orc, base, model)
    say(f"full-model sensitivity {base} {model}")
    assert rel(host(G.sensitivity()), orc.sensitivity(g)) <= 1e-5


@pytest.mark.parametrize("base,model", CASES)
def test_projections(pet, orc, base, model):
    G, g, d, _ = make(pet, orc, base, model)
    rng = np.random.default_rng(1)
    f = f32(rng.uniform(0.5, 2.0, G.img_shape))
    w = f32(rng.uniform(-1.0, 1.0, G.sino_shape))
    M = d["n_subsets"]
    for subset in ([0, 1, M] if base != "c2" else [0, 7]):
        say(f"full-model forward/back {base} {model} subset {subset}")
        q = host(G.forward(dev(f), subset))
        qo = orc.forward(g, f, subset)
        mask = np.zeros(G.sino_shape, bool)
        for a in range(d["n_angles"]):
            if subset == 0 or a % M == subset - 1:
                mask[:, a] = True
        assert rel(q[mask], qo[mask]) <= 1e-5, (subset, rel(q[mask], qo[mask]))
        b = host(G.back(dev(w), subset))
        assert rel(b, orc.back(g, w, subset)) <= 1e-5


@pytest.mark.parametrize("base,model", [("c1", "full"), ("ragged", "full8")])
def test_adjoint_identity(pet, orc, base, model):
    G, _, _, _ = make(pet, orc, base, model)
    rng = np.random.default_rng(3)
    x = dev(rng.uniform(0, 1, G.img_shape))
    yv = dev(rng.normal(0, 1, G.sino_shape))
    Ax = G.forward(x, 0)
    ATy = G.back(yv, 0)
    lhs = float((Ax.double() * yv.double()).sum())
    rhs = float((x.double() * ATy.double()).sum())
    scale = float((Ax.double().abs() * yv.double().abs()).sum())
    assert abs(lhs - rhs) <= 1e-5 * scale


@pytest.mark.parametrize("base,ns", [("c1", 32), ("ragged", 8), ("c2", 32)])
def test_attenuation_factors(pet, orc, base, ns):
    """exp(-line integrals of mu) through the sub-ray model, no PSF."""
    d = full_desc(dict(BASE[base], n_subrays=ns, psf_fwhm=6.59))
    G = pet.Geometry(d)
    mu = f32(support_mu(d))
    att = host(G.attenuation_factors(dev(mu)))
    g = orc.geom(dict(d, psf_fwhm=0.0))
    ref = np.exp(-orc.forward(g, mu))
    assert rel(att, ref) <= 1e-6
    assert att.min() > 0.0 and att.max() <= 1.0


def one_step(pet, orc, G, g, p, f, y, r, k, i, t_nest=1.0):
    st = pet.State(G, p)
    st.seek(k, i, t_nest)
    fg = dev(f)
    st.subiteration(fg, dev(y), dev(r))
    st.close()
    rec = orc.Recon(g, orc.params(p), f, y, r)
    rec.st.k, rec.st.i, rec.st.t_nest = k, i, t_nest
    rec.subiteration()
    return host(fg), rec.image()


@pytest.mark.parametrize("base,model", [("c1", "full"), ("ragged", "full8"), ("c2", "full")])
def test_subiteration_from_oracle_state(pet, orc, base, model):
    """One GPU subiteration (SDP-P2 with computed nu, and OSEM) from FP32
    inputs along the oracle's own OSEM trajectory."""
    from oracle import osem as O
    from synth import configs
    G, g, d, _ = make(pet, orc, base, model)
    f0, y, r = data(orc, g, d, 5)
    M = d["n_subsets"]
    f = f32(O.osem(g, f0, y, r, 1))             # a realistic iterate
    p = configs.params_2d(M, 1e7, mode="P2", U=1e4)
    p.update(J0=0)
    for (k, i) in [(0, 1), (1, 2), (3, M)]:
        say(f"full-model subiteration {base} {model} P2 k={k} i={i}")
        gpu, ref = one_step(pet, orc, G, g, p, f, y, r, k, i)
        assert rel(gpu, ref) <= 1e-5, (k, i, rel(gpu, ref))
    say(f"full-model subiteration {base} {model} OSEM")
    i = 2 if M > 1 else 1
    st = pet.State(G, pet.osem_params())
    st.seek(0, i, 1.0)
    fg = dev(f)
    st.subiteration(fg, dev(y), dev(r))
    st.close()
    assert rel(host(fg), O.osem_subiteration(g, f, y, r, i)) <= 1e-5


@pytest.mark.parametrize("base,model", [("c1", "full"), ("ragged", "full8")])
def test_subset_gradient_and_objective(pet, orc, base, model):
    from oracle import gradcons as gc
    G, g, d, _ = make(pet, orc, base, model)
    f0, y, r = data(orc, g, d, 6)
    rng = np.random.default_rng(7)
    f = f32(rng.uniform(0.5, 2.0, G.img_shape))
    p = dict(mode="P2", beta=0.3, gamma_R=2.0, eps=1e-12, t_clip=1e-4, U=1e4, lambda0=1.0, a=0.1, rho=3.0,
             delta1=2.0, delta2=2.0, nu1=0.5, nu2=2.0, J0=3, J1=1000)
    from tests.test_gpu_gradcons import magnitude_bound
    for subset in (0, 1):
        hg = host(G.subset_gradient(p, dev(f), dev(y), dev(r), subset))
        ho = gc.subset_gradient(g, f, y, r, subset, p["beta"], p["gamma_R"], p["eps"])
        bound = magnitude_bound(orc, g, f, y, r, subset, p)
        e = float(np.linalg.norm(hg - ho) / np.linalg.norm(bound))
        assert e <= 1e-5, (subset, e)
    phi = G.objective(p, dev(f), dev(y), dev(r))
    assert phi == pytest.approx(orc.objective(g, f, y, r, p["beta"], p["gamma_R"], p["eps"]), rel=1e-6)


def test_full_model_rejected_by_batch(pet, orc):
    G, _, d, _ = make(pet, orc, "c1", "full")
    from synth import configs
    b = pet.Batch(2)
    z = torch.ones(G.img_shape, device="cuda")
    s = torch.ones(G.sino_shape, device="cuda")
    with pytest.raises(pet.PetOSError):
        b.add(G, configs.params_2d(4, 1e5, U=10.0), z, s, s, 1)
    b.close()
