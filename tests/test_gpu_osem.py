"""GPU parity of the OSEM initialisation (Hudson-Larkin; Sec. IV-C) through
the C ABI against the FP64 oracle: one subiteration from the same FP32 input
(rel-L2 <= 1e-5, the projectors' bar), two full iterations as the paper uses
them (<= 1e-4: the EM update is a contraction-free product of ratios, so the
FP32 errors of the 2M subiterations add up without being amplified), and
the OSEM-then-SDP composition."""
import numpy as np
import pytest

from tests.test_gpu_parity import dev, f32, full_desc, host, rel, say, workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = ["c1", "ragged_aniso", "odd_angles", "3d_small", "3d_ragged", "c2"]


@pytest.fixture(scope="module")
def pet():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2111_07886_amd as pet
    pet.lib()
    return pet


@pytest.mark.parametrize("name", CASES)
def test_osem_one_subiteration(pet, orc, name):
    from oracle import osem as O
    w, _, _ = workload(name, orc)
    g = orc.geom(w.desc)
    G = pet.Geometry(full_desc(w.desc))
    M = w.desc["n_subsets"]
    y, r = f32(w.y), f32(w.r)
    rng = np.random.default_rng(11)
    f = f32(rng.uniform(0.5, 2.0, G.img_shape))
    st = pet.State(G, pet.osem_params())
    for i in ([1, 2, M] if M > 2 else [1, M]):
        st.seek(0, i, 1.0)
        say(f"osem {name} subset {i}")
        fg = dev(f)
        st.subiteration(fg, dev(y), dev(r))
        ref = O.osem_subiteration(g, f, y, r, i)
        e = rel(host(fg), ref)
        assert e <= 1e-5, (i, e)
    st.close()


@pytest.mark.parametrize("name", CASES)
def test_osem_two_iterations(pet, orc, name):
    from oracle import osem as O
    w, _, _ = workload(name, orc)
    g = orc.geom(w.desc)
    G = pet.Geometry(full_desc(w.desc))
    y, r = f32(w.y), f32(w.r)
    say(f"osem 2 iterations {name}")
    fg = dev(w.f0)
    pet.reconstruct(G, pet.osem_params(), fg, dev(y), dev(r), 2)
    ref = O.osem(g, w.f0, y, r, 2)
    e = rel(host(fg), ref)
    say(f"  rel-L2 {e:.2e}")
    assert e <= 1e-4


def test_osem_then_sdp_composition(pet, orc):
    """reconstruct_osem_init = an OSEM state for n_osem iterations followed by
    pet_os_reconstruct from its image (bitwise), and the objective it reaches
    is below that of the same SDP iterations from f0 = 1."""
    w, p, _ = workload("c1", orc)
    G = pet.Geometry(full_desc(w.desc))
    y, r = dev(w.y), dev(w.r)
    f1 = dev(w.f0)
    pet.reconstruct_osem_init(G, p, f1, y, r, 2, 3)
    f2 = dev(w.f0)
    st = pet.State(G, pet.osem_params(p["beta"], p["gamma_R"], p["eps"]))
    st.run(f2, y, r, 2)
    st.close()
    pet.reconstruct(G, p, f2, y, r, 3)
    assert torch.equal(f1, f2)
    f3 = dev(w.f0)
    pet.reconstruct(G, p, f3, y, r, 3)
    assert G.objective(p, f1, y, r) < G.objective(p, f3, y, r)


def test_osem_rejected_by_batch_and_server(pet):
    w, _, _ = workload("c1", None)
    G = pet.Geometry(full_desc(w.desc))
    b = pet.Batch(2)
    with pytest.raises(pet.PetOSError):
        b.add(G, pet.osem_params(), dev(w.f0), dev(w.y), dev(w.r), 2)
    b.close()
