"""The boundary's data check on the GPU: the problem statement of Sec. II-A
(counts g >= 0, background gamma > 0 elementwise) and the box B of
eq:BoundedSet (0 <= f0 <= U), every value finite.  Each reconstruction entry
point rejects data that break a rule with INVALID_ARG before queuing any work
(the caller's image is unchanged); a batch and a server keep running their
other requests, whose results stay bitwise equal to their solo results.  A
corrupted checkpoint is rejected without touching the state."""
import struct

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu-boundary] {msg}", flush=True)


@pytest.fixture(scope="module")
def pet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_07886_amd as pet
    pet.lib()
    return pet


def dev(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda").contiguous()


def small_2d(seed=41):
    from synth import configs, phantoms
    d = configs.desc_2d(48, 32, 71, 2.5, 4)
    w = phantoms.make_2d(d, seed=seed, n_ell=4, counts=2e5, bg_frac=0.1)
    return w, configs.params_2d(4, 2e5, U=w.U)


def small_3d(seed=42):
    from synth import configs, phantoms
    d = configs.desc_3d(24, 8, 16, 37, 2.5, 3.0, 8, 3, 4)
    w = phantoms.make_3d(d, seed=seed, n_ell=3, counts=1e6, bg_uniform=0.15, bg_scatter=0.15,
                         scatter_sigma_bins=4.0)
    return w, configs.params_3d(U=w.U)


def corruptions(w, p):
    """(label, f0, y, r, params) cases that break one rule each."""
    f0, y, r = w.f0.copy(), w.y.copy(), w.r.copy()
    out = []
    yb = y.copy(); yb.reshape(-1)[7] = np.nan
    out.append(("y NaN", f0, yb, r, p))
    yb = y.copy(); yb.reshape(-1)[3] = -1.0
    out.append(("y < 0", f0, yb, r, p))
    rb = r.copy(); rb.reshape(-1)[11] = 0.0
    out.append(("r = 0", f0, y, rb, p))
    rb = r.copy(); rb.reshape(-1)[-1] = np.inf
    out.append(("r inf", f0, y, rb, p))
    fb = f0.copy(); fb.reshape(-1)[5] = -0.5
    out.append(("f0 < 0", fb, y, r, p))
    fb = f0.copy(); fb.reshape(-1)[9] = 2.0 * p["U"]
    out.append(("f0 > U", fb, y, r, p))
    out.append(("f0 = 0, adaptive nu from J = 1", np.zeros_like(f0), y, r, dict(p, mode="P2", J0=0)))
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_reconstruct_rejects_bad_data(pet, dim):
    w, p = small_2d() if dim == 2 else small_3d()
    G = pet.Geometry(w.desc)
    for label, f0, y, r, pp in corruptions(w, p):
        say(f"reconstruct {dim}D: {label}")
        f = dev(f0)
        keep = f.clone()
        with pytest.raises(pet.PetOSError) as e:
            pet.reconstruct(G, pp, f, dev(y), dev(r), 1)
        assert e.value.code == -1, label
        torch.cuda.synchronize()
        assert torch.equal(f, keep), label                  # nothing was queued
    # the clean data pass, and an image at U itself is in B
    f0 = w.f0.copy()
    f0.reshape(-1)[0] = float(np.float32(p["U"])) if float(np.float32(p["U"])) <= p["U"] else 0.0
    pet.reconstruct(G, p, dev(f0), dev(w.y), dev(w.r), 1)


def test_state_checks_each_new_triple(pet):
    w, p = small_2d()
    G = pet.Geometry(w.desc)
    st = pet.State(G, p)
    y, r, f = dev(w.y), dev(w.r), dev(w.f0)
    rb = w.r.copy(); rb.reshape(-1)[0] = -1.0
    rbad = dev(rb)
    with pytest.raises(pet.PetOSError) as e:
        st.subiteration(f, y, rbad)
    assert e.value.code == -1 and st.position() == (0, 1)
    with pytest.raises(pet.PetOSError):
        st.run(f, y, rbad, 1)
    assert st.position() == (0, 1)
    st.subiteration(f, y, r)                  # the same state with clean data
    assert st.position() == (0, 2)


def test_3d_state_follows_new_data_buffers(pet):
    """A 3D state reads y and r from a bin-major copy made when it first sees
    a (y, r) pair of buffers: a new pair mid-reconstruction is copied and
    used.  The second subiteration with new counts equals, bit for bit, that
    of a state sought to the same position from the same image, and differs
    from a second subiteration with the old counts."""
    w, p = small_3d()
    G = pet.Geometry(w.desc)
    y, r, f0 = dev(w.y), dev(w.r), dev(w.f0)
    y2 = dev(2.0 * w.y)
    st = pet.State(G, p)
    f = f0.clone()
    st.subiteration(f, y, r)
    f1 = f.clone()
    st.subiteration(f, y2, r)                  # new counts, new buffer
    fa = f.clone()
    old = pet.State(G, p)
    g = f0.clone()
    old.subiteration(g, y, r)
    old.subiteration(g, y, r)                  # the old counts again
    fresh = pet.State(G, p)
    fresh.seek(0, 2)
    h = f1.clone()
    fresh.subiteration(h, y2, r)
    say(f"3D new data buffers: |a - fresh| = {float((fa - h).abs().max())}, |a - old| = {float((fa - g).abs().max())}")
    assert torch.equal(fa, h)
    assert not torch.equal(fa, g)


def test_batch_add_rejects_bad_data(pet):
    w, p = small_2d(43)
    G = pet.Geometry(w.desc)
    y, r = dev(w.y), dev(w.r)
    solo = dev(w.f0)
    pet.reconstruct(G, p, solo, y, r, 2)
    B = pet.Batch(4)
    f = dev(w.f0)
    B.add(G, p, f, y, r, 2)
    yb = w.y.copy(); yb.reshape(-1)[1] = np.nan
    fb = dev(w.f0)
    with pytest.raises(pet.PetOSError) as e:
        B.add(G, p, fb, dev(yb), r, 2)
    assert e.value.code == -1
    B.run()
    torch.cuda.synchronize()
    assert torch.equal(f, solo)
    assert torch.equal(fb, dev(w.f0))
    B.close()


def test_server_fails_only_bad_requests(pet, tmp_path, monkeypatch):
    """A served mix of clean 2D/3D requests and requests with a NaN count, a
    zero background or an image above U: the bad ones end with INVALID_ARG
    (nothing run), the clean ones equal their solo results bitwise."""
    monkeypatch.setenv("PET_OS_TUNE_CACHE", str(tmp_path / "tune.txt"))
    clean = [small_2d(50), small_2d(51), small_3d(52), small_2d(53)]
    solo = []
    for w, p in clean:
        G = pet.Geometry(w.desc)
        pet.autotune(G)
        f = dev(w.f0)
        pet.reconstruct(G, p, f, dev(w.y), dev(w.r), 2)
        solo.append(f)
    torch.cuda.synchronize()
    wb, pb = small_2d(54)
    yb = wb.y.copy(); yb.reshape(-1)[2] = np.nan
    rb = wb.r.copy(); rb.reshape(-1)[5] = 0.0
    fb = wb.f0.copy(); fb.reshape(-1)[0] = 3.0 * pb["U"]
    bad = [(wb, pb, wb.f0, yb, wb.r), (wb, pb, wb.f0, wb.y, rb), (wb, pb, fb, wb.y, wb.r)]
    S = pet.Server(4 << 30, 3)
    jobs = []
    for k in range(4):
        w, p = clean[k]
        data = (dev(w.f0), dev(w.y), dev(w.r))
        jobs.append(("clean", k, data, S.submit(w.desc, p, *data, n_iter=2, want_objective=True)))
        if k < 3:
            w, p, f0, y, r = bad[k]
            data = (dev(f0), dev(y), dev(r))
            jobs.append(("bad", k, data, S.submit(w.desc, p, *data, n_iter=2)))
    res = [(kind, k, data, S.wait(t)) for kind, k, data, t in jobs]
    S.close()
    for kind, k, data, r in res:
        say(f"served {kind} {k}: status {r['status']} {r['message']}")
        if kind == "bad":
            assert r["status"] == -1 and r["subiterations"] == 0, (k, r)
        else:
            assert r["status"] == 0, (k, r)
            assert torch.equal(data[0], solo[k]), k


def test_import_rejects_corrupt_checkpoint(pet):
    """pet_os_state_import validates the parameters, the Nesterov t and the
    frozen-nu flag before writing anything: the state keeps its position."""
    w, p = small_2d()
    G = pet.Geometry(w.desc)
    y, r = dev(w.y), dev(w.r)
    f = dev(w.f0)
    src = pet.State(G, p)
    for _ in range(3):
        src.subiteration(f, y, r)
    blob = bytearray(src.export())
    # header layout: magic[8], version u32, have_frozen u32, descriptor, params, k i64, i i32, pad, t_nest f64
    import ctypes as C
    off_desc = 16
    off_params = off_desc + C.sizeof(pet.GeomDesc)
    off_params = (off_params + 7) // 8 * 8
    off_U = off_params + pet.Params.U.offset
    off_k = off_params + C.sizeof(pet.Params)
    off_k = (off_k + 7) // 8 * 8
    off_t = off_k + 16
    assert struct.unpack_from("<d", blob, off_U)[0] == p["U"]
    assert struct.unpack_from("<q", blob, off_k)[0] == 0 and struct.unpack_from("<i", blob, off_k + 8)[0] == 4
    dst = pet.State(G, p)
    dst.subiteration(f, y, r)
    cases = {"U <= 0": (off_U, "<d", -1.0), "t_nest < 1": (off_t, "<d", 0.5),
             "t_nest NaN": (off_t, "<d", float("nan"))}
    for label, (off, fmt, val) in cases.items():
        bad = bytearray(blob)
        struct.pack_into(fmt, bad, off, val)
        with pytest.raises(pet.PetOSError) as e:
            dst.import_(bytes(bad))
        assert e.value.code == -1, label
        assert dst.position() == (0, 2), label
    # a frozen-nu flag for a mode that holds no nu
    pb = dict(p, mode="BSREM")
    s_b = pet.State(G, pb)
    blob_b = bytearray(s_b.export())
    struct.pack_into("<I", blob_b, 12, 1)
    with pytest.raises(pet.PetOSError) as e:
        pet.State(G, pb).import_(bytes(blob_b))
    assert e.value.code == -1
    dst.import_(bytes(blob))
    assert dst.position() == (0, 4)
