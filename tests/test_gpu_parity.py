"""GPU parity: every kernel of the hot path, called through the C ABI, against
the FP64 oracle on the same FP32 inputs.

Tolerances: rel-L2 <= 1e-5 per projection (forward, back, sensitivity, one
subiteration), <= 1e-4 on the image after the configured iterations, <= 1e-6
relative on the objective."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu-parity] {msg}", flush=True)


@pytest.fixture(scope="module")
def pet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_07886_amd as pet
    pet.lib()
    return pet


def dev(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


GEOMS = {
    "c1": dict(dim=2, nx=64, ny=64, vx=2.0, vy=2.0, n_angles=60, n_radial=95, ds=2.0, n_subsets=4),
    "ragged_aniso": dict(dim=2, nx=50, ny=37, vx=2.0, vy=2.5, n_angles=30, n_radial=71, ds=1.7, n_subsets=5),
    "odd_angles": dict(dim=2, nx=41, ny=41, vx=1.5, vy=1.5, n_angles=45, n_radial=61, ds=1.5, n_subsets=9),
    "even_bins": dict(dim=2, nx=32, ny=32, vx=2.0, vy=2.0, n_angles=16, n_radial=46, ds=2.0, n_subsets=16),
    "c2": dict(dim=2, nx=256, ny=256, vx=300 / 256, vy=300 / 256, n_angles=288, n_radial=367,
               ds=300 / 256, n_subsets=24),
    "3d_small": dict(dim=3, nx=24, ny=20, nz=8, vx=2.5, vy=2.5, vz=3.0, n_angles=16, n_radial=33, ds=2.5,
                     n_rings=8, max_ring_diff=3, ring_pitch=3.0, det_radius=120.0, n_subsets=4),
    "3d_ragged": dict(dim=3, nx=35, ny=35, nz=13, vx=2.0, vy=2.0, vz=2.5, n_angles=24, n_radial=49, ds=2.0,
                      n_rings=13, max_ring_diff=5, ring_pitch=2.5, det_radius=150.0, n_subsets=6),
    # direct planes only (one ring difference), an odd depth
    "3d_d0": dict(dim=3, nx=17, ny=12, nz=5, vx=2.0, vy=2.0, vz=2.5, n_angles=10, n_radial=25, ds=2.0,
                  n_rings=5, max_ring_diff=0, ring_pitch=2.5, det_radius=120.0, n_subsets=2),
    # 33 ring differences: more than the column-staging forward projector
    # takes, so the per-wave one runs
    "3d_many_d": dict(dim=3, nx=20, ny=18, nz=40, vx=2.0, vy=2.0, vz=2.5, n_angles=12, n_radial=31, ds=2.0,
                      n_rings=40, max_ring_diff=16, ring_pitch=2.5, det_radius=150.0, n_subsets=4),
}


def full_desc(d):
    d = dict(d)
    d.setdefault("nz", 1)
    d.setdefault("vz", 1.0)
    d.setdefault("n_rings", 1)
    d.setdefault("max_ring_diff", 0)
    d.setdefault("ring_pitch", 1.0)
    d.setdefault("det_radius", 0.0)
    return d


@pytest.fixture(scope="module")
def geoms(pet, orc):
    out = {}
    for k, d in GEOMS.items():
        d = full_desc(d)
        say(f"create geometry {k}")
        out[k] = (pet.Geometry(d), orc.geom(d), d)
    return out


@pytest.mark.parametrize("name", list(GEOMS))
def test_sensitivity(geoms, orc, name):
    G, g, _ = geoms[name]
    say(f"sensitivity {name}")
    s = host(G.sensitivity())
    so = orc.sensitivity(g)
    assert rel(s, so) <= 1e-5


@pytest.mark.parametrize("name", list(GEOMS))
def test_forward_projection(geoms, orc, name):
    G, g, _ = geoms[name]
    rng = np.random.default_rng(1)
    f = f32(rng.uniform(0.5, 2.0, G.img_shape))
    subsets = [0, 1, g.n_subsets] if name != "c2" else [0, 7]
    for subset in subsets:
        say(f"forward {name} subset {subset}")
        q = host(G.forward(dev(f), subset))
        qo = orc.forward(g, f, subset)
        mask = np.zeros(G.sino_shape, bool)
        for a in range(g.n_angles):
            if subset == 0 or a % g.n_subsets == subset - 1:
                mask[:, a] = True
        assert rel(q[mask], qo[mask]) <= 1e-5, (subset, rel(q[mask], qo[mask]))


@pytest.mark.parametrize("name", ["3d_small", "3d_ragged", "3d_d0", "3d_many_d"])
def test_nnz_3d(geoms, orc, name):
    """Nonzeros of A (counting pieces, no image read) against the oracle's
    traces over every ray of subset 1, and the subsets adding up to the whole.
    Crossings through a cell corner leave the FP64 trace pieces of length
    ~1e-14 mm; the FP32 fractions keep some of them, so the count lies
    between the oracle's pieces longer than 1e-9 mm and its pieces of any
    positive length (plus a margin for corners the FP32 fractions split)."""
    G, g, d = geoms[name]
    say(f"nnz {name}")
    total = G.nnz(0)
    parts = [G.nnz(s) for s in range(1, d["n_subsets"] + 1)]
    assert sum(parts) == total
    n_pos = n_real = 0
    for a in range(0, d["n_angles"], d["n_subsets"]):
        for plane in range(orc.n_planes(g)):
            for b in range(d["n_radial"]):
                _, ln = orc.trace(g, plane, a, b)
                n_pos += int(np.count_nonzero(ln > 0.0))
                n_real += int(np.count_nonzero(ln > 1e-9))
    say(f"nnz {name}: {parts[0]} against {n_real} .. {n_pos}")
    assert n_real <= parts[0] <= n_pos + 1e-3 * n_real, (parts[0], n_real, n_pos)


@pytest.mark.parametrize("name", list(GEOMS))
def test_back_projection(geoms, orc, name):
    G, g, _ = geoms[name]
    rng = np.random.default_rng(2)
    w = f32(rng.uniform(-1.0, 1.0, G.sino_shape))
    for subset in [0, 2]:
        say(f"back {name} subset {subset}")
        b = host(G.back(dev(w), subset))
        bo = orc.back(g, w, subset)
        assert rel(b, bo) <= 1e-5, (subset, rel(b, bo))


@pytest.mark.parametrize("name", ["c1", "ragged_aniso", "3d_ragged"])
def test_gpu_adjoint_identity(geoms, name):
    G, g, _ = geoms[name]
    rng = np.random.default_rng(3)
    x = dev(rng.uniform(0, 1, G.img_shape))
    yv = dev(rng.normal(0, 1, G.sino_shape))
    say(f"adjoint {name}")
    Ax = G.forward(x, 0)
    ATy = G.back(yv, 0)
    lhs = float((Ax.double() * yv.double()).sum())
    rhs = float((x.double() * ATy.double()).sum())
    scale = float((Ax.double().abs() * yv.double().abs()).sum())
    assert abs(lhs - rhs) <= 1e-5 * scale


def workload(name, orc):
    from synth import configs, phantoms
    if name == "c1":
        return configs.c1()
    if name == "c2":
        return configs.c2()
    if name == "3d_small":
        d = full_desc(GEOMS["3d_small"])
        w = phantoms.make_3d(d, seed=21, n_ell=4, counts=2e6, bg_uniform=0.15, bg_scatter=0.15,
                             scatter_sigma_bins=4.0)
        return w, configs.params_3d(U=w.U), 3
    if name == "3d_ragged":
        d = full_desc(GEOMS["3d_ragged"])
        w = phantoms.make_3d(d, seed=22, n_ell=5, counts=5e6, bg_uniform=0.15, bg_scatter=0.15,
                             scatter_sigma_bins=4.0)
        return w, configs.params_3d(U=w.U), 2
    d = full_desc(GEOMS[name])
    w = phantoms.make_2d(d, seed=23, n_ell=5, counts=3e5, bg_frac=0.1)
    return w, configs.params_2d(d["n_subsets"], 3e5, U=w.U), 4


def stepwise(pet, orc, w, p, samples, tol=1e-5, tune=False, branches=None, label=None):
    """One GPU subiteration from the oracle's own state (iterate cast to FP32,
    position, Nesterov t, frozen nu) at each sampled J, against one oracle
    subiteration from the same FP32 input (tune: shapes from the autotuner).
    branches: a dict that receives, over the samples, the number of voxels
    whose entering value takes the upper branch of S (f >= U/2,
    eq:preconditioner) and the number the oracle's P_t sends to U - t or to t
    (eq:OperatorPt)."""
    G = pet.Geometry(full_desc(w.desc))
    if tune:
        pet.autotune(G)
    st = pet.State(G, p)
    y, r = dev(w.y), dev(w.r)
    rec = orc.Recon(orc.geom(w.desc), orc.params(p), w.f0, host(y), host(r))
    worst = 0.0
    U, t = p["U"], p["t_clip"]
    for J in range(1, max(samples) + 1):
        if J in samples:
            fin = f32(rec.f)
            ref = rec.clone_with(fin)
            ref.frozen = f32(rec.frozen)
            ref.subiteration()
            nu = dev(ref.frozen.reshape(G.img_shape)) if rec.st.have_frozen else None
            st.seek(rec.st.k, rec.st.i, rec.st.t_nest, nu)
            fg = dev(fin.reshape(G.img_shape))
            st.subiteration(fg, y, r)
            got = host(fg)
            e = rel(got, ref.image())
            worst = max(worst, e)
            assert e <= tol, (J, e)
            if branches is not None:
                fo = ref.image().reshape(-1)
                branches["upper"] = branches.get("upper", 0) + int((fin >= 0.5 * U).sum())
                branches["clamp_hi"] = branches.get("clamp_hi", 0) + int((fo == U - t).sum())
                branches["clamp_lo"] = branches.get("clamp_lo", 0) + int((fo == t).sum())
                # the voxels the GPU sends to U - t (FP32 value of U - t); P_t
                # decides on f~, which FP32 and FP64 round differently, so a
                # voxel may be clamped on one side only when the other side's
                # value lies within rounding of the threshold U
                hi = float(np.float32(U - t))
                gv = got.reshape(-1)
                gh = gv == hi
                oh = fo == U - t
                branches["clamp_hi_gpu"] = branches.get("clamp_hi_gpu", 0) + int(gh.sum())
                branches["clamp_hi_differ"] = branches.get("clamp_hi_differ", 0) + int((gh != oh).sum())
                near = 1e-5 * U
                assert np.all(fo[gh & ~oh] >= U - t - near), (J, fo[gh & ~oh])
                assert np.all(gv[oh & ~gh] >= U - t - near), (J, gv[oh & ~gh])
        rec.subiteration()
    from parity_record import record
    label = label or f"{w.desc['dim']}D {w.desc['nx']}x{w.desc['ny']}x{w.desc.get('nz', 1)} {p['mode']}"
    record("stepwise", label,
           samples=len(samples), worst_rel_l2=worst, tol=tol, U=U, **(branches or {}))
    return worst


@pytest.mark.parametrize("mode", ["BSREM", "M1", "M2", "P1", "P2"])
def test_stepwise_c1_every_subiteration(pet, orc, mode):
    """C1 workload, every one of its 40 subiterations, with J0 = 2 and J1 = 6
    so that nu = 1, adaptive nu, the freeze and frozen nu are all exercised."""
    from synth import configs
    w, _, n_iter = configs.c1()
    p = configs.params_2d(4, 1e5, mode=mode, U=w.U)
    p.update(J0=2, J1=6)
    say(f"stepwise C1 {mode}")
    worst = stepwise(pet, orc, w, p, set(range(1, 4 * n_iter + 1)), label=f"C1 {mode}")
    say(f"stepwise C1 {mode}: worst one-step rel-L2 {worst:.2e}")


SMALL_U = 2.0   # U as a multiple of max f_true: iterates cross U/2 and reach U


@pytest.mark.parametrize("kind", [0, 1])
def test_stepwise_small_U_2d(pet, orc, tmp_path, monkeypatch, kind):
    """The upper branch of S (eq:preconditioner: (U - f)/p for f >= U/2) and
    the upper clamp of P_t (eq:OperatorPt: f~ >= U gives U - t) on the GPU:
    the 64^2 workload in SDP-P2 with U = 2 max f_true, every subiteration of
    its 10 iterations from the oracle's state, with each back-projector tile
    (16x16; 8x8 with four angle groups) pinned through the tuning cache."""
    from synth import configs
    w, _, n_iter = configs.c1()
    U = SMALL_U * float(w.f_true.max())
    p = configs.params_2d(4, 1e5, mode="P2", U=U)
    p.update(J0=2, J1=6)
    d = full_desc(w.desc)
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{tune_key(d)}|16 {kind}\n")
    monkeypatch.setenv("PET_OS_TUNE_CACHE", str(cache))
    say(f"stepwise small U 2D kind {kind}")
    br = {}
    worst = stepwise(pet, orc, w, p, set(range(1, 4 * n_iter + 1)), tune=True, branches=br,
                     label=f"C1 P2 U = 2 max f, tile kind {kind}")
    say(f"stepwise small U 2D kind {kind}: worst {worst:.2e}, branches {br}")
    assert br["upper"] > 100 and br["clamp_hi"] > 10 and br["clamp_hi_gpu"] > 10


@pytest.mark.parametrize("name", ["3d_small", "3d_ragged"])
def test_stepwise_small_U_3d(pet, orc, name):
    """As above on the 3D update kernel (U = 2 max f_true, SDP-P2 of Table III)."""
    from synth import configs
    w, _, n_iter = workload(name, orc)
    p = configs.params_3d(U=SMALL_U * float(w.f_true.max()))
    M = w.desc["n_subsets"]
    say(f"stepwise small U {name}")
    br = {}
    worst = stepwise(pet, orc, w, p, set(range(1, n_iter * M + 1)), branches=br, label=f"{name} P2 U = 2 max f")
    say(f"stepwise small U {name}: worst {worst:.2e}, branches {br}")
    assert br["upper"] > 100 and br["clamp_hi"] > 5 and br["clamp_hi_gpu"] > 5


def test_box_clamps_decide_as_fp64(pet, orc):
    """P_t (eq:OperatorPt) compares the FP32 step result with U as the FP64
    comparison does, also for a U that is not a float.  With a vanishing
    step (lambda0 = 1e-30) f~ = f exactly on both sides, so a voxel at the
    float 3.0 just below U = 3 + 2^-30 is kept (rounding U to the nearest
    float would clamp it to U - t), a voxel at 0 goes to t, and every voxel
    of the GPU result equals the oracle's rounded to FP32."""
    from synth import configs
    w, _, _ = configs.c1()
    U = 3.0 + 2.0 ** -30
    assert float(np.float32(U)) == 3.0 < U
    p = configs.params_2d(4, 1e5, mode="BSREM", U=U)
    p.update(lambda0=1e-30)
    f0 = np.full(w.f0.shape, 1.0)
    f0[20:40, 10:50] = 3.0
    f0[41:44, 10:50] = 0.0
    f0[45:48, 10:50] = float(np.nextafter(np.float32(1.5), np.float32(0)))
    G = pet.Geometry(full_desc(w.desc))
    y, r = dev(w.y), dev(w.r)
    st = pet.State(G, p)
    fg = dev(f0)
    st.subiteration(fg, y, r)
    ref = orc.Recon(orc.geom(w.desc), orc.params(p), f32(f0), host(y), host(r))
    ref.subiteration()
    got, fo = host(fg).reshape(-1), ref.f
    assert np.all(fo[(f0 == 3.0).reshape(-1)] == 3.0)
    assert np.all(fo[(f0 == 0.0).reshape(-1)] == p["t_clip"])
    assert np.array_equal(got, f32(fo))


def test_stepwise_c2_full_size(pet, orc):
    """C2 at full size (256^2, 288 x 367, 24 subsets, P2) along its whole 1,200
    subiteration trajectory: every subiteration of the first two iterations,
    then samples through the nu freeze at J1 = 1000 and to the end."""
    from synth import configs
    w, p, n_iter = configs.c2()
    samples = set(range(1, 49)) | {97, 240, 480, 720, 960, 999, 1000, 1001, 1002, 1100, 1199, 1200}
    say("stepwise C2")
    worst = stepwise(pet, orc, w, p, samples, label="C2 256^2 P2")
    say(f"stepwise C2: worst one-step rel-L2 {worst:.2e}")


@pytest.mark.parametrize("name", ["ragged_aniso", "odd_angles", "even_bins", "3d_small", "3d_ragged"])
def test_stepwise_other_geometries(pet, orc, name):
    w, p, n_iter = workload(name, orc)
    M = w.desc["n_subsets"]
    say(f"stepwise {name}")
    stepwise(pet, orc, w, p, set(range(1, n_iter * M + 1)))


NOISE = 5e-7   # size of the FP32 evaluation error of one subiteration (stepwise tests: 1e-7 .. 1e-6)


def intrinsic_spread(orc, w, p, n_iter, seeds=(0, 1), per_iteration=False):
    """Sensitivity of the method itself: the FP64 oracle against the same FP64
    oracle perturbed after every subiteration by relative noise of the size of
    one FP32 subiteration's evaluation error.  Returns the largest image
    rel-L2 and objective relative difference after n_iter iterations (with
    per_iteration, the objective's after each of the n_iter iterations, as a
    list)."""
    g, P = orc.geom(w.desc), orc.params(p)
    y, r = f32(w.y), f32(w.r)
    M = w.desc["n_subsets"]
    clean = orc.Recon(g, P, w.f0, y, r)
    phis = []
    for k in range(n_iter):
        for _ in range(M):
            clean.subiteration()
        if per_iteration or k == n_iter - 1:
            phis.append(clean.objective())
    e_img, e_obj = 0.0, [0.0] * len(phis)
    for sd in seeds:
        rng = np.random.default_rng(sd)
        noisy = orc.Recon(g, P, w.f0, y, r)
        n_obj = 0
        for k in range(n_iter):
            for _ in range(M):
                noisy.subiteration()
                noisy.f *= 1.0 + NOISE * rng.standard_normal(noisy.f.shape)
            if per_iteration or k == n_iter - 1:
                e_obj[n_obj] = max(e_obj[n_obj], abs(noisy.objective() - phis[n_obj]) / abs(phis[n_obj]))
                n_obj += 1
        e_img = max(e_img, rel(noisy.f, clean.f))
    return e_img, (e_obj if per_iteration else e_obj[-1])


TOL_IMG, TOL_OBJ = 1e-4, 1e-6    # stated: image after the configured iterations, objective
IMG_PARITY_LIMIT = 1e-2           # above this a widened image tolerance pins nothing: not asserted


def check_trajectory(pet, orc, w, p, n_iter, label):
    """Image after the configured iterations and the objective against the
    oracle's trajectory.  The tolerance applied is the stated one (1e-4 image,
    1e-6 objective) or, where the method itself separates two trajectories
    by more (measured on the oracle: FP64 against FP64 perturbed by noise of
    the size of one FP32 subiteration's error), 5x that spread.  An image
    tolerance widened beyond 1e-2 would pin nothing, so such an image is only
    recorded (the stepwise tests are that workload's parity evidence); the
    objective is asserted in every case.  Each case is recorded
    (parity_record) with its errors, spreads and applied tolerances."""
    from parity_record import record
    G = pet.Geometry(full_desc(w.desc))
    f = dev(w.f0)
    y, r = dev(w.y), dev(w.r)
    say(f"trajectory {label}")
    obj = pet.reconstruct(G, p, f, y, r, n_iter, want_objective=True)
    fo, objo = orc.reconstruct(orc.geom(w.desc), orc.params(p), w.f0, host(y), host(r), n_iter)
    e = rel(host(f), fo)
    eo = abs(obj[-1] - objo[-1]) / abs(objo[-1])
    s_img, s_obj = intrinsic_spread(orc, w, p, n_iter)
    tol_img = max(TOL_IMG, 5.0 * s_img)
    tol_obj = max(TOL_OBJ, 5.0 * s_obj)
    img_asserted = tol_img <= IMG_PARITY_LIMIT
    say(f"trajectory {label}: image rel-L2 {e:.2e} (spread {s_img:.2e}, tol {tol_img:.1e}"
        f"{'' if img_asserted else ', not asserted'}); objective {eo:.2e} (spread {s_obj:.2e}, tol {tol_obj:.1e})")
    record("trajectory", label, n_iter=n_iter, image_rel_l2=e, image_spread=s_img, image_tol=tol_img,
           image_face_value=tol_img == TOL_IMG, image_asserted=img_asserted, objective_rel=eo,
           objective_spread=s_obj, objective_tol=tol_obj, objective_face_value=tol_obj == TOL_OBJ,
           mode=p["mode"])
    if img_asserted:
        assert e <= tol_img
    assert eo <= tol_obj
    return e, s_img


@pytest.mark.parametrize("mode", ["BSREM", "M1", "M2", "P1", "P2"])
def test_c1_trajectory_all_modes(pet, orc, mode):
    from synth import configs
    w, _, n_iter = configs.c1()
    check_trajectory(pet, orc, w, configs.params_2d(4, 1e5, mode=mode, U=w.U), n_iter, f"C1 {mode}")


@pytest.mark.parametrize("name", ["ragged_aniso", "odd_angles", "even_bins", "3d_small", "3d_ragged"])
def test_trajectory_other_geometries(pet, orc, name):
    w, p, n_iter = workload(name, orc)
    check_trajectory(pet, orc, w, p, n_iter, name)


def test_c2_full_trajectory(pet, orc):
    """The 256^2 / 288 x 367 / 24-subset workload, all 50 iterations (1,200
    subiterations, nu frozen at J = 1000), in the launch configuration the
    benchmark times."""
    from synth import configs
    w, p, n_iter = configs.c2()
    check_trajectory(pet, orc, w, p, n_iter, "C2")


def test_determinism_and_reconstruct_equals_subiterations(pet):
    from synth import configs
    w, p, _ = configs.c1()
    G = pet.Geometry(full_desc(w.desc))
    y, r = dev(w.y), dev(w.r)
    f1, f2, f3 = dev(w.f0), dev(w.f0), dev(w.f0)
    say("determinism")
    pet.reconstruct(G, p, f1, y, r, 3)
    pet.reconstruct(G, p, f2, y, r, 3)
    st = pet.State(G, p)
    for _ in range(12):
        st.subiteration(f3, y, r)
    torch.cuda.synchronize()
    assert torch.equal(f1, f2)
    assert torch.equal(f1, f3)


def test_checkpoint_resume_bitwise(pet):
    from synth import configs
    w, p, _ = configs.c1()
    p = dict(p, J0=1, J1=5)
    G = pet.Geometry(full_desc(w.desc))
    y, r = dev(w.y), dev(w.r)
    fa, fb = dev(w.f0), dev(w.f0)
    say("checkpoint")
    sa = pet.State(G, p)
    for _ in range(16):
        sa.subiteration(fa, y, r)
    sb = pet.State(G, p)
    for _ in range(7):
        sb.subiteration(fb, y, r)
    blob = sb.export()
    sb.close()
    sc = pet.State(G, p)
    sc.import_(blob)
    assert sc.position() == (1, 4)
    for _ in range(9):
        sc.subiteration(fb, y, r)
    torch.cuda.synchronize()
    assert torch.equal(fa, fb)
    other = pet.State(pet.Geometry(full_desc(GEOMS["even_bins"])), configs.params_2d(16, 1e5, U=w.U))
    with pytest.raises(pet.PetOSError) as e:
        other.import_(blob)
    assert e.value.code == -7


@pytest.mark.parametrize("name", ["c1", "3d_ragged"])
def test_objective_and_default_U(pet, orc, name):
    """The FP64 objective (eq:ObjectiveFunction: the forward projector's
    log-likelihood epilogue and the RDP sum) and the default U, in 2D and
    with the 3D forward projector's staged columns."""
    w, p, _ = workload(name, orc)
    G = pet.Geometry(full_desc(w.desc))
    g = orc.geom(w.desc)
    rng = np.random.default_rng(4)
    f = f32(rng.uniform(0.2, 3.0, G.img_shape))
    y, r = dev(w.y), dev(w.r)
    say(f"objective/default U {name}")
    phi = G.objective(p, dev(f), y, r)
    phio = orc.objective(g, f, host(y), host(r), p["beta"], p["gamma_R"], p["eps"])
    assert abs(phi - phio) <= 1e-6 * abs(phio)
    U = G.default_U(dev(f), y, r)
    Uo = orc.default_U(g, f, host(y), host(r))
    assert abs(U - Uo) <= 1e-5 * Uo


def test_edge_subset_counts(pet, orc):
    """M = 1 (one subset holds every angle) and M = n_angles (one angle each)."""
    from synth import phantoms, configs
    for M in (1, 16):
        d = full_desc(dict(GEOMS["even_bins"], n_subsets=M))
        w = phantoms.make_2d(d, seed=31, n_ell=3, counts=1e5, bg_frac=0.1)
        p = configs.params_2d(M, 1e5, U=w.U)
        say(f"edge M={M}")
        stepwise(pet, orc, w, p, set(range(1, 2 * M + 1)))
        check_trajectory(pet, orc, w, p, 2, f"edge M={M}")


def test_invalid_params_rejected(pet):
    from synth import configs
    G = pet.Geometry(full_desc(GEOMS["even_bins"]))
    base = configs.params_2d(16, 1e5)
    for bad in (dict(eps=0.0), dict(t_clip=2e6), dict(nu1=3.0), dict(J0=5, J1=2), dict(a=-1.0),
                dict(mode=7), dict(beta=-0.1)):
        with pytest.raises(pet.PetOSError) as e:
            pet.State(G, dict(base, **bad))
        assert e.value.code == -1
    f = torch.ones(G.img_shape, device="cuda")
    with pytest.raises(ValueError):
        G.forward(torch.ones(5, device="cuda"))
    with pytest.raises(TypeError):
        G.forward(f.double())
    assert math.isfinite(G.objective(base, f, torch.ones(G.sino_shape, device="cuda"),
                                     torch.ones(G.sino_shape, device="cuda")))


def test_c3_full_size(pet, orc):
    """The fully 3D 200x200x64 / 224 x 281 x 1744-plane / 28-subset workload at
    full size: one subset's forward and back-projection, then one subiteration
    from the oracle's state at J = 1 and J = 2 (rel-L2 <= 1e-5 each)."""
    from synth import configs
    w, p, _ = configs.c3()
    d = full_desc(w.desc)
    G, g = pet.Geometry(d), orc.geom(d)
    rng = np.random.default_rng(7)
    f = f32(rng.uniform(0.5, 2.0, G.img_shape))
    say("C3 forward subset 5")
    q = host(G.forward(dev(f), 5))
    qo = orc.forward(g, f, 5)
    sub = [a for a in range(g.n_angles) if a % g.n_subsets == 4]
    assert rel(q[:, sub], qo[:, sub]) <= 1e-5
    del q, qo
    say("C3 back subset 11")
    wv = f32(rng.uniform(-1.0, 1.0, G.sino_shape))
    b = host(G.back(dev(wv), 11))
    bo = orc.back(g, wv, 11)
    assert rel(b, bo) <= 1e-5
    del wv, b, bo
    say("C3 stepwise J = 1, 2")
    stepwise(pet, orc, w, p, {1, 2})


# 3D with ragged 8x8 column tiles (27 x 21) and a depth (40) that no z-block
# size divides; span of slice offsets 4, so every staging shape but
# (64 slices, 8 ring differences) fits the back-projector's LDS
GEOM_Z = dict(dim=3, nx=27, ny=21, nz=40, vx=2.0, vy=2.0, vz=2.5, n_angles=16, n_radial=39, ds=2.0,
              n_rings=40, max_ring_diff=2, ring_pitch=2.5, det_radius=150.0, n_subsets=4)


def tune_key(d):
    """The tuning cache's key of a descriptor (the library's format)."""
    return "%d %d %d %d %.17g %.17g %.17g %d %d %.17g %d %d %.17g %.17g %d" % (
        d["dim"], d["nx"], d["ny"], d["nz"], d["vx"], d["vy"], d["vz"], d["n_angles"], d["n_radial"], d["ds"],
        d["n_rings"], d["max_ring_diff"], d["ring_pitch"], d["det_radius"], d["n_subsets"])


@pytest.mark.parametrize("zb,dpg", [(16, 4), (16, 8), (32, 4), (32, 8), (64, 4)])
def test_bp3_shapes(pet, orc, tmp_path, monkeypatch, zb, dpg):
    """Every slices-per-block / ring-differences-per-group shape the 3D
    autotuner can choose, pinned through its cache file: the subset
    back-projection and fused subiterations against the oracle."""
    from synth import configs, phantoms
    d = full_desc(GEOM_Z)
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{tune_key(d)}|0 {zb * 16 + dpg}\n")
    monkeypatch.setenv("PET_OS_TUNE_CACHE", str(cache))
    say(f"bp3 shape zb={zb} dpg={dpg}")
    G = pet.Geometry(d)
    pet.autotune(G)
    assert cache.read_text().count("|") == 1          # the cached shape was taken, not retuned
    sh = G.shapes()
    assert (sh["current"]["bp3_zb"], sh["current"]["bp3_dpg"]) == (zb, dpg)
    assert sh["current"]["bp_kind"] == sh["default"]["bp_kind"] == 2 and sh["default"]["bp3_zb"] == 64
    g = orc.geom(d)
    rng = np.random.default_rng(zb + dpg)
    wv = f32(rng.uniform(-1.0, 1.0, G.sino_shape))
    assert rel(host(G.back(dev(wv), 2)), orc.back(g, wv, 2)) <= 1e-5
    ones = np.ones(G.sino_shape)
    assert rel(host(G.back(dev(ones), 0)), orc.back(g, ones, 0)) <= 1e-5     # every angle
    w = phantoms.make_3d(d, seed=31, n_ell=4, counts=2e6, bg_uniform=0.15, bg_scatter=0.15, scatter_sigma_bins=4.0)
    stepwise(pet, orc, w, configs.params_3d(U=w.U), {1, 2, 5}, tune=True)


@pytest.mark.parametrize("seg", [1, 4, 16, 64])
@pytest.mark.parametrize("kind", [0, 1])
def test_2d_shapes(pet, orc, tmp_path, monkeypatch, seg, kind):
    """Every 2D shape the autotuner can choose (forward threads per ray x
    back-projector tile), pinned through its cache file, against the oracle
    on a ragged anisotropic geometry: subset forward and back-projection and
    fused subiterations."""
    from synth import phantoms, configs
    d = full_desc(GEOMS["ragged_aniso"])
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{tune_key(d)}|{seg} {kind}\n")
    monkeypatch.setenv("PET_OS_TUNE_CACHE", str(cache))
    say(f"2d shape seg={seg} kind={kind}")
    G = pet.Geometry(d)
    pet.autotune(G)
    assert cache.read_text().count("|") == 1          # the cached shape was taken, not retuned
    assert G.shapes()["current"]["fp_seg"] == seg and G.shapes()["current"]["bp_kind"] == kind
    g = orc.geom(d)
    rng = np.random.default_rng(seg * 2 + kind)
    f = f32(rng.uniform(0.5, 2.0, G.img_shape))
    sub = [a for a in range(g.n_angles) if a % g.n_subsets == 2]
    assert rel(host(G.forward(dev(f), 3))[:, sub], orc.forward(g, f, 3)[:, sub]) <= 1e-5
    wv = f32(rng.uniform(-1.0, 1.0, G.sino_shape))
    assert rel(host(G.back(dev(wv), 3)), orc.back(g, wv, 3)) <= 1e-5
    w = phantoms.make_2d(d, seed=23, n_ell=5, counts=3e5, bg_frac=0.1)
    stepwise(pet, orc, w, configs.params_2d(d["n_subsets"], 3e5, U=w.U), {1, 2, 7}, tune=True)


@pytest.mark.parametrize("name", ["ragged_aniso", "c2"])
def test_forward_sum_independent_of_threads_per_ray(pet, tmp_path, monkeypatch, name):
    """A ray's sum is cut into fixed leaves added by a fixed tree, so every
    threads-per-ray shape gives the same bits (which lets a batch choose its
    own shape and still compute what each request computes alone)."""
    d = full_desc(GEOMS[name])
    rng = np.random.default_rng(9)
    f = dev(rng.uniform(0.5, 2.0, (d["ny"], d["nx"])))
    out = []
    for seg in (1, 4, 16, 64):
        cache = tmp_path / f"tune{seg}.txt"
        cache.write_text(f"{tune_key(d)}|{seg} 0\n")
        monkeypatch.setenv("PET_OS_TUNE_CACHE", str(cache))
        G = pet.Geometry(d)
        pet.autotune(G)
        assert G.shapes()["current"]["fp_seg"] == seg
        out.append(G.forward(f, 0))
    torch.cuda.synchronize()
    for k in range(1, 4):
        assert torch.equal(out[0], out[k]), k


def test_invalid_cached_shape_is_retuned(pet, tmp_path, monkeypatch):
    """A cache entry naming a shape the tuner cannot choose is ignored."""
    d = full_desc(GEOMS["ragged_aniso"])
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{tune_key(d)}|7 1\n")
    monkeypatch.setenv("PET_OS_TUNE_CACHE", str(cache))
    G = pet.Geometry(d)
    pet.autotune(G)
    assert G.shapes()["current"]["fp_seg"] in (1, 4, 16, 64)
    assert cache.read_text().count("|") == 2          # retuned and stored
