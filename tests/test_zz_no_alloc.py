"""pet_os_reconstruct_noalloc, through the C ABI, against pet_os_reconstruct
(the entry point it varies): the same iterations with the scratch in the
library's static device array give the same image bit for bit.  Several calls
in a row reuse the array, each smaller than the one before it, so what a call
leaves there must not leak into the next; a request whose scratch exceeds the
array is rejected and changes nothing."""
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


def cases():
    """Largest first: the 64^2 workload (SDP-P2, nu adaptive then frozen),
    a 3D request, then a 2D one on fewer voxels (BSREM)."""
    from synth import configs, phantoms
    w1, p1, _ = configs.c1()
    p1 = dict(p1, J0=1, J1=5)
    d3 = configs.desc_3d(24, 6, 16, 37, 2.5, 3.0, 6, 3, 4)
    w3 = phantoms.make_3d(d3, seed=61, n_ell=3, counts=1e6, bg_uniform=0.15, bg_scatter=0.15,
                          scatter_sigma_bins=4.0)
    d2 = configs.desc_2d(40, 30, 61, 3.0, 5)
    w2 = phantoms.make_2d(d2, seed=62, n_ell=4, counts=2e5, bg_frac=0.1)
    return [("64x64 P2", w1, p1, 3), ("24x24x6 P2", w3, configs.params_3d(U=w3.U), 2),
            ("40x40 BSREM", w2, configs.params_2d(5, 2e5, mode="BSREM", U=w2.U), 3)]


def test_noalloc_equals_reconstruct(pet):
    cs = cases()
    sizes = [w.f0.size for _, w, _, _ in cs]
    assert sizes == sorted(sizes, reverse=True)            # each call smaller than the one before
    for rep in range(2):                                   # the whole sequence twice
        for label, w, p, n in cs:
            print(f"[no-alloc] {label}, pass {rep}", flush=True)
            G = pet.Geometry(w.desc)
            y, r = dev(w.y), dev(w.r)
            ref = dev(w.f0)
            pet.reconstruct(G, p, ref, y, r, n)
            f = dev(w.f0)
            pet.reconstruct_noalloc(G, p, f, y, r, n)
            torch.cuda.synchronize()
            assert torch.equal(f, ref), label
            assert not torch.equal(f, dev(w.f0)), label    # the iterations ran


def test_noalloc_fits_the_3d_workload(pet):
    """The static area holds a 200x200x64 request with 224 x 281 x 1744 bins
    and 28 subsets (synthetic data: one iteration runs)."""
    from synth import configs
    d = configs.desc_3d(200, 64, 224, 281, 1.5, 3.0, 64, 15, 28)
    G = pet.Geometry(d)
    p = configs.params_3d(U=1e6)
    f = torch.ones(G.img_shape, device="cuda")
    y = torch.ones(G.sino_shape, device="cuda")
    r = torch.ones(G.sino_shape, device="cuda")
    pet.reconstruct_noalloc(G, p, f, y, r, 1)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(f).all()) and not bool((f == 1.0).all())


def test_noalloc_rejects_what_does_not_fit(pet):
    from synth import configs
    # three 4096^2 images of scratch (gradient, mu, snapshot): 192 MiB > 96 MiB
    d = configs.desc_2d(4096, 4, 9, 0.1, 2)
    G = pet.Geometry(d)
    p = configs.params_2d(2, 1e5, mode="BSREM")
    f = torch.ones(G.img_shape, device="cuda")
    y = torch.ones(G.sino_shape, device="cuda")
    r = torch.ones(G.sino_shape, device="cuda")
    with pytest.raises(pet.PetOSError) as e:
        pet.reconstruct_noalloc(G, p, f, y, r, 1)
    assert e.value.code == -1 and "static area" in str(e.value)
    torch.cuda.synchronize()
    assert bool((f == 1.0).all())
    # OSEM needs a state's subset sensitivities
    with pytest.raises(pet.PetOSError):
        pet.reconstruct_noalloc(G, pet.osem_params(), f, y, r, 1)
