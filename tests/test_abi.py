"""The C-ABI library loads on a host without a GPU, exports every function
that include/pet_os.h declares, and rejects invalid arguments before it
touches the device (no GPU needed for any call made here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pet_os.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pet_os_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def pet():
    import paper_2111_07886_amd as pet
    if not os.path.exists(pet.LIB_PATH):
        from paper_2111_07886_amd import build
        build.build()
    pet.lib()
    return pet


def test_exports_every_declared_symbol(pet):
    decl = declared_functions()
    assert len(decl) >= 15
    lib = C.CDLL(pet.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(pet.EXPORTS) == decl


def test_version_string(pet):
    assert b"gfx950" in pet.lib().pet_os_version()


def _desc(**kw):
    d = dict(dim=2, nx=16, ny=16, nz=1, vx=2.0, vy=2.0, vz=1.0, n_angles=12, n_radial=25, ds=2.0,
             n_rings=1, max_ring_diff=0, ring_pitch=1.0, det_radius=0.0, n_subsets=4)
    d.update(kw)
    return d


@pytest.mark.parametrize("bad", [dict(dim=4), dict(nx=0), dict(nx=1 << 23, ny=1), dict(vx=-1.0), dict(ds=float("nan")),
                                 dict(n_subsets=0), dict(n_subsets=13), dict(n_angles=0),
                                 dict(dim=3, nz=8, vz=3.0, n_rings=7, ring_pitch=3.0, max_ring_diff=2,
                                      det_radius=300.0),
                                 dict(dim=3, nz=8, vz=3.0, n_rings=8, ring_pitch=3.0, max_ring_diff=2,
                                      det_radius=10.0),
                                 dict(dim=3, nz=8, vz=3.0, n_rings=8, ring_pitch=3.0, max_ring_diff=8,
                                      det_radius=300.0)])
def test_invalid_geometry_rejected_before_device(pet, bad):
    d = pet.desc_struct(_desc(**bad))
    h = C.c_void_p()
    rc = pet.lib().pet_os_create_geometry(C.byref(d), C.byref(h))
    assert rc == -1
    assert h.value is None
    assert pet.last_error()


def test_3d_strides_limited_to_24_bit_products(pet):
    # the forward projector multiplies voxel strides in 24-bit integers
    d = pet.desc_struct(_desc(dim=3, nx=1 << 17, ny=1, nz=64, vz=3.0, n_rings=64, ring_pitch=3.0,
                              max_ring_diff=2, det_radius=3e5))
    h = C.c_void_p()
    assert pet.lib().pet_os_create_geometry(C.byref(d), C.byref(h)) == -1
    assert h.value is None
    assert "2^23" in pet.last_error()


def test_null_arguments(pet):
    L = pet.lib()
    assert L.pet_os_create_geometry(None, None) == -1
    assert L.pet_os_destroy_geometry(None) == -1
    assert L.pet_os_state_create(None, None, None) == -1
    assert L.pet_os_subiteration(None, None, None, None, None) == -1
    assert L.pet_os_reconstruct(None, None, None, None, None, 1, None, None) == -1
    assert L.pet_os_state_export(None, None, None) == -1
    assert "NULL" in pet.last_error()
