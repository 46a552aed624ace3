"""Served mode on the GPU: requests of different sizes (2D and 3D) arriving
while others run are admitted into the running batch, and each result is
the same as the request's solo pet_os_reconstruct result (bitwise: same
kernels, same reductions, same tuned shapes via the shared tuning cache)."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_07886_amd as pet
    pet.lib()
    return pet


def dev(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda").contiguous()


def test_served_results_equal_solo(pet, tmp_path, monkeypatch):
    from synth import configs, phantoms
    monkeypatch.setenv("PET_OS_TUNE_CACHE", str(tmp_path / "tune.txt"))
    trace = configs.c5_trace(n_requests=40, rate=400.0, seed=77)
    reqs = []
    for q in trace[:14]:
        d = q["desc"]
        if d["dim"] == 3:
            d = configs.desc_3d(32, 8, 24, 49, 300.0 / 128, 300.0 / 128, 8, 3, 4)
            w = phantoms.make_3d(d, seed=q["seed"], n_ell=3, counts=1e6, bg_uniform=0.1, bg_scatter=0.1,
                                 scatter_sigma_bins=4.0)
            p = configs.params_3d(U=w.U)
        else:
            w = phantoms.make_2d(d, seed=q["seed"], n_ell=6, counts=q["counts"], bg_frac=0.2)
            p = configs.params_2d(d["n_subsets"], q["counts"], U=w.U)
        reqs.append((w, p, 2, q["arrival_s"]))
    if not any(w.desc["dim"] == 3 for w, *_ in reqs):
        d = configs.desc_3d(32, 8, 24, 49, 300.0 / 128, 300.0 / 128, 8, 3, 4)
        w = phantoms.make_3d(d, seed=5, n_ell=3, counts=1e6, bg_uniform=0.1, bg_scatter=0.1, scatter_sigma_bins=4.0)
        reqs.append((w, configs.params_3d(U=w.U), 2, reqs[-1][3]))
    # solo references
    solo = []
    for w, p, n, _ in reqs:
        G = pet.Geometry(w.desc)
        pet.autotune(G)
        f = dev(w.f0)
        pet.reconstruct(G, p, f, dev(w.y), dev(w.r), n)
        solo.append(f)
    torch.cuda.synchronize()
    S = pet.Server(8 << 30, 5)          # fewer slots than requests: queueing and joining
    data = [(dev(w.f0), dev(w.y), dev(w.r)) for w, *_ in reqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = []
    for (w, p, n, at), (f, y, r) in zip(reqs, data):
        dt = at - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(S.submit(w.desc, p, f, y, r, n, want_objective=True))
    res = [S.wait(t) for t in tickets]
    st = S.stats()
    S.close()
    assert all(r["status"] == 0 for r in res), [(k, r["status"], r["message"]) for k, r in enumerate(res)
                                                if r["status"] != 0]
    assert st["max_active"] > 1
    for k, ((f, _, _), ref) in enumerate(zip(data, solo)):
        assert torch.equal(f, ref), k
    for (w, p, n, _), r, ref in zip(reqs, res, solo):
        G = pet.Geometry(w.desc)
        phi = G.objective(p, ref, dev(w.y), dev(w.r))
        assert abs(r["objective"] - phi) <= 1e-12 * abs(phi)
