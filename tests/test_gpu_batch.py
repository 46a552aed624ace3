"""Batched execution (pet_os_batch_*, pet_os_reconstruct_batch): uneven
requests advanced together by one captured launch sequence per subiteration
compute exactly what each computes alone (bitwise), and agree with the FP64
oracle; slots can join and leave between steps; graph replays stay correct
with eager work in between."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu-batch] {msg}", flush=True)


@pytest.fixture(scope="module")
def pet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_07886_amd as pet
    pet.lib()
    return pet


def dev(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda").contiguous()


def requests(n=7, seed=5):
    """Uneven 2D requests shaped like the batched workload (sizes, angles,
    subsets, counts), small enough for the oracle, plus one 3D request."""
    import math
    from synth import configs, phantoms
    rng = np.random.default_rng(seed)
    out = []
    modes = ["BSREM", "M1", "M2", "P1", "P2"]
    for k in range(n):
        nn = int(rng.choice([32, 48, 64, 80]))
        M = int(rng.integers(2, 9))
        Na = max(2 * M, (int(rng.integers(20, 61)) // M) * M)
        Nr = 2 * int(math.ceil(nn / math.sqrt(2))) + 3
        d = configs.desc_2d(nn, Na, Nr, 128.0 / nn, M)
        counts = float(10 ** rng.uniform(5, 6.5))
        w = phantoms.make_2d(d, seed=900 + k, n_ell=4, counts=counts, bg_frac=0.1)
        p = configs.params_2d(M, counts, mode=modes[k % 5], U=w.U)
        out.append((w, p, int(rng.integers(2, 5))))
    d3 = configs.desc_3d(24, 8, 16, 37, 2.5, 3.0, 8, 3, 4)
    w3 = phantoms.make_3d(d3, seed=950, n_ell=3, counts=1e6, bg_uniform=0.15, bg_scatter=0.15, scatter_sigma_bins=4.0)
    out.append((w3, configs.params_3d(U=w3.U), 2))
    return out


def test_batch_equals_alone_bitwise(pet, orc):
    reqs = requests()
    geoms = [pet.Geometry(w.desc) for w, _, _ in reqs]
    ys = [dev(w.y) for w, _, _ in reqs]
    rs = [dev(w.r) for w, _, _ in reqs]
    alone = []
    for (w, p, n), G, y, r in zip(reqs, geoms, ys, rs):
        f = dev(w.f0)
        pet.reconstruct(G, p, f, y, r, n)
        alone.append(f)
    fs = [dev(w.f0) for w, _, _ in reqs]
    say(f"reconstruct_batch of {len(reqs)}")
    pet.reconstruct_batch(geoms, [p for _, p, _ in reqs], fs, ys, rs, [n for _, _, n in reqs])
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(alone, fs)):
        assert torch.equal(a, b), k
    # one request against the oracle (well-conditioned BSREM member)
    w, p, n = reqs[0]
    fo, _ = orc.reconstruct(orc.geom(w.desc), orc.params(p), w.f0, ys[0].cpu().double().numpy(),
                            rs[0].cpu().double().numpy(), n, want_obj=False)
    e = np.linalg.norm(fs[0].cpu().double().numpy() - fo) / np.linalg.norm(fo)
    say(f"request 0 ({p['mode']}) vs oracle rel-L2 {e:.2e}")
    assert e <= 1e-4


def test_slots_join_and_leave(pet):
    """Continuous batching: a request added while others are mid-way, and a
    slot reused after removal, still compute exactly their solo result."""
    reqs = requests(n=4, seed=6)[:4]
    geoms = [pet.Geometry(w.desc) for w, _, _ in reqs]
    ys = [dev(w.y) for w, _, _ in reqs]
    rs = [dev(w.r) for w, _, _ in reqs]
    alone = []
    for (w, p, n), G, y, r in zip(reqs, geoms, ys, rs):
        f = dev(w.f0)
        pet.reconstruct(G, p, f, y, r, n)
        alone.append(f)
    fs = [dev(w.f0) for w, _, _ in reqs]
    B = pet.Batch(3)
    s0 = B.add(geoms[0], reqs[0][1], fs[0], ys[0], rs[0], reqs[0][2])
    s1 = B.add(geoms[1], reqs[1][1], fs[1], ys[1], rs[1], reqs[1][2])
    B.step(3)
    s2 = B.add(geoms[2], reqs[2][1], fs[2], ys[2], rs[2], reqs[2][2])    # joins mid-way
    B.run()
    torch.cuda.synchronize()
    for s in (s0, s1, s2):
        assert B.status(s) == (False, 0)
    B.remove(s1)
    s3 = B.add(geoms[3], reqs[3][1], fs[3], ys[3], rs[3], reqs[3][2])    # reuses a slot
    assert s3 == s1
    B.run()
    torch.cuda.synchronize()
    for k in range(4):
        assert torch.equal(alone[k], fs[k]), k
    assert B.bytes() > 0
    B.close()


def test_graph_replays_with_eager_work_between(pet):
    """The captured step is replayed many times with unrelated eager work and
    synchronisations in between; every replay matches the solo path."""
    reqs = requests(n=3, seed=7)[:3]
    geoms = [pet.Geometry(w.desc) for w, _, _ in reqs]
    ys = [dev(w.y) for w, _, _ in reqs]
    rs = [dev(w.r) for w, _, _ in reqs]
    fs = [dev(w.f0) for w, _, _ in reqs]
    solo = [dev(w.f0) for w, _, _ in reqs]
    states = [pet.State(G, p) for G, (_, p, _) in zip(geoms, reqs)]
    B = pet.Batch(4)
    for k, ((w, p, n), G) in enumerate(zip(reqs, geoms)):
        B.add(G, p, fs[k], ys[k], rs[k], n)
    junk = torch.zeros(1 << 20, device="cuda")
    for step in range(6):
        B.step(1)
        junk.add_(1.0)                       # eager work between replays
        torch.cuda.synchronize()
        for k in range(3):
            if step < reqs[k][2] * reqs[k][0].desc["n_subsets"]:
                states[k].subiteration(solo[k], ys[k], rs[k])
        torch.cuda.synchronize()
        for k in range(3):
            assert torch.equal(fs[k], solo[k]), (step, k)
    B.close()


def test_autotune_keeps_results(pet, tmp_path, monkeypatch):
    """Autotuned shapes change the launch configuration, not the iterate beyond
    FP32 summation order; the choice is cached by descriptor."""
    monkeypatch.setenv("PET_OS_TUNE_CACHE", str(tmp_path / "tune.txt"))
    w, p, n = requests(n=1, seed=8)[0]
    G = pet.Geometry(w.desc)
    y, r = dev(w.y), dev(w.r)
    f1 = dev(w.f0)
    pet.reconstruct(G, p, f1, y, r, n)
    pet.autotune(G, force=True)
    f2 = dev(w.f0)
    pet.reconstruct(G, p, f2, y, r, n)
    torch.cuda.synchronize()
    e = float((f1.double() - f2.double()).norm() / f1.double().norm())
    assert e <= 1e-4
    assert (tmp_path / "tune.txt").read_text().count("|") == 1
    G2 = pet.Geometry(w.desc)
    pet.autotune(G2)                          # from the cache
    f3 = dev(w.f0)
    pet.reconstruct(G2, p, f3, y, r, n)
    torch.cuda.synchronize()
    assert torch.equal(f2, f3)
