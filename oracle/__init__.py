"""FP64 CPU oracle of SDP-BSREM (Guo et al., arXiv 2111.07886).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the product package.
It shares no code with the HIP path.  ``build()`` compiles ``oracle.c`` with
gcc (-O2, no fast-math, OpenMP) into ``liboracle.so`` next to this file.

Thin ctypes wrapper: numpy float64 arrays in, numpy arrays out.  Every
routine it wraps names its equation in ``oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODES = {"BSREM": 0, "M1": 1, "M2": 2, "P1": 3, "P2": 4}


def build(force: bool = True) -> str:
    """Compile the oracle shared library (gcc, FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("vx", C.c_double), ("vy", C.c_double), ("vz", C.c_double),
                ("n_angles", C.c_int), ("n_radial", C.c_int), ("ds", C.c_double),
                ("n_rings", C.c_int), ("max_ring_diff", C.c_int),
                ("ring_pitch", C.c_double), ("det_radius", C.c_double),
                ("n_subsets", C.c_int), ("n_sub", C.c_int), ("psf_fwhm", C.c_double),
                ("att", C.POINTER(C.c_double))]


class _Params(C.Structure):
    _fields_ = [("mode", C.c_int), ("beta", C.c_double), ("gamma_R", C.c_double),
                ("eps", C.c_double), ("t_clip", C.c_double), ("U", C.c_double),
                ("lambda0", C.c_double), ("a", C.c_double), ("rho", C.c_double),
                ("delta1", C.c_double), ("delta2", C.c_double), ("nu1", C.c_double),
                ("nu2", C.c_double), ("J0", C.c_long), ("J1", C.c_long)]


class _State(C.Structure):
    _fields_ = [("k", C.c_long), ("i", C.c_int), ("t_nest", C.c_double),
                ("have_frozen", C.c_int)]


_lib = None
_D = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        G, P, S = C.POINTER(_Geom), C.POINTER(_Params), C.POINTER(_State)
        sig = {
            "orc_n_planes": (C.c_int, [G]), "orc_n_voxels": (C.c_int, [G]),
            "orc_n_bins": (C.c_long, [G]),
            "orc_plane_rings": (None, [G, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "orc_angle": (None, [G, C.c_int, _D, _D]),
            "orc_trace": (C.c_int, [G, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), _D, C.c_int]),
            "orc_chord_clip": (C.c_double, [G, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
            "orc_chord_clip_off": (C.c_double, [G, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                                C.c_int]),
            "orc_trace_off": (C.c_int, [G, C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_int), _D,
                                        C.c_int]),
            "orc_subray_offset": (C.c_double, [G, C.c_int]),
            "orc_blur": (None, [G, _D, _D]),
            "orc_psf_radius": (C.c_int, [G, C.c_double]),
            "orc_forward": (None, [G, _D, C.c_int, _D]),
            "orc_back": (None, [G, _D, C.c_int, _D]),
            "orc_sensitivity": (None, [G, _D]),
            "orc_precond_norm": (None, [G, _D, _D]),
            "orc_rdp_value": (C.c_double, [G, _D, C.c_double, C.c_double]),
            "orc_rdp_grad": (None, [G, _D, C.c_double, C.c_double, _D]),
            "orc_rdp_hess_apply": (None, [G, _D, C.c_double, C.c_double, _D, _D]),
            "orc_grad_mag": (None, [G, _D, _D]),
            "orc_fidelity": (C.c_double, [G, _D, _D, _D]),
            "orc_objective": (C.c_double, [G, _D, _D, _D, C.c_double, C.c_double, C.c_double]),
            "orc_relax": (C.c_double, [P, C.c_long]),
            "orc_nesterov_next": (C.c_double, [C.c_double]),
            "orc_km_alpha": (C.c_double, [P, C.c_long]),
            "orc_default_U": (C.c_double, [G, _D, _D, _D]),
            "orc_state_init": (None, [S]),
            "orc_subiteration": (C.c_int, [G, P, S, _D, _D, _D, _D, _D, _D]),
            "orc_reconstruct": (C.c_int, [G, P, _D, _D, _D, C.c_int, _D]),
            "orc_num_threads": (C.c_int, []),
            "orc_set_num_threads": (None, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def geom(desc: dict) -> _Geom:
    """Oracle geometry from a descriptor dict (same keys as the C-ABI desc)."""
    g = _Geom()
    g.dim = int(desc["dim"])
    g.nx, g.ny = int(desc["nx"]), int(desc["ny"])
    g.nz = int(desc.get("nz", 1)) if g.dim == 3 else 1
    g.vx, g.vy = float(desc["vx"]), float(desc["vy"])
    g.vz = float(desc.get("vz", 1.0))
    g.n_angles, g.n_radial = int(desc["n_angles"]), int(desc["n_radial"])
    g.ds = float(desc["ds"])
    g.n_rings = int(desc.get("n_rings", 1))
    g.max_ring_diff = int(desc.get("max_ring_diff", 0))
    g.ring_pitch = float(desc.get("ring_pitch", g.vz))
    g.det_radius = float(desc.get("det_radius", 0.0))
    g.n_subsets = int(desc["n_subsets"])
    g.n_sub = int(desc.get("n_subrays", 1))
    g.psf_fwhm = float(desc.get("psf_fwhm", 0.0))
    if desc.get("att") is not None:
        # the factors live as long as the geometry object
        g._att = np.ascontiguousarray(np.asarray(desc["att"], dtype=np.float64).reshape(-1))
        g.att = g._att.ctypes.data_as(C.POINTER(C.c_double))
    if g.dim == 3 and (g.n_rings != g.nz or g.ring_pitch != g.vz):
        raise ValueError("oracle: rings must sit at slice centres (n_rings == nz, ring_pitch == vz)")
    return g


def params(p: dict) -> _Params:
    q = _Params()
    q.mode = MODES[p["mode"]] if isinstance(p["mode"], str) else int(p["mode"])
    for k in ("beta", "gamma_R", "eps", "t_clip", "U", "lambda0", "a", "rho",
              "delta1", "delta2", "nu1", "nu2"):
        setattr(q, k, float(p[k]))
    q.J0, q.J1 = int(p["J0"]), int(p["J1"])
    return q


def n_planes(g): return _load().orc_n_planes(C.byref(g))
def n_voxels(g): return _load().orc_n_voxels(C.byref(g))
def n_bins(g): return _load().orc_n_bins(C.byref(g))
def num_threads(): return _load().orc_num_threads()
def set_num_threads(n): _load().orc_set_num_threads(int(n))


def sino_shape(g):
    return (n_planes(g), g.n_angles, g.n_radial)


def img_shape(g):
    return (g.nz, g.ny, g.nx) if g.dim == 3 else (g.ny, g.nx)


def plane_rings(g, plane):
    r1, r2 = C.c_int(), C.c_int()
    _load().orc_plane_rings(C.byref(g), plane, C.byref(r1), C.byref(r2))
    return r1.value, r2.value


def angle(g, a):
    c, s = C.c_double(), C.c_double()
    _load().orc_angle(C.byref(g), a, C.byref(c), C.byref(s))
    return c.value, s.value


def trace(g, plane, a, b):
    cap = 2 * (g.nx + g.ny + g.nz) + 8
    vox = (C.c_int * cap)()
    ln = np.zeros(cap)
    n = _load().orc_trace(C.byref(g), plane, a, b, vox, _ptr(ln), cap)
    return np.array(vox[:n], dtype=np.int64), ln[:n].copy()


def chord_clip(g, plane, a, b, ix, iy, iz=0):
    return _load().orc_chord_clip(C.byref(g), plane, a, b, ix, iy, iz)


def chord_clip_off(g, plane, a, b, off, ix, iy, iz=0):
    return _load().orc_chord_clip_off(C.byref(g), plane, a, b, off, ix, iy, iz)


def subray_offset(g, k):
    return _load().orc_subray_offset(C.byref(g), k)


def blur(g, f):
    f = _f64(f).reshape(-1)
    out = np.zeros_like(f)
    _load().orc_blur(C.byref(g), _ptr(f), _ptr(out))
    return out.reshape(img_shape(g))


def psf_radius(g, v):
    return _load().orc_psf_radius(C.byref(g), v)


def forward(g, f, subset=0):
    f = _f64(f).reshape(-1)
    q = np.zeros(n_bins(g))
    _load().orc_forward(C.byref(g), _ptr(f), subset, _ptr(q))
    return q.reshape(sino_shape(g))


def back(g, w, subset=0):
    w = _f64(w).reshape(-1)
    out = np.zeros(n_voxels(g))
    _load().orc_back(C.byref(g), _ptr(w), subset, _ptr(out))
    return out.reshape(img_shape(g))


def sensitivity(g):
    s = np.zeros(n_voxels(g))
    _load().orc_sensitivity(C.byref(g), _ptr(s))
    return s.reshape(img_shape(g))


def precond_norm(g, s):
    s = _f64(s).reshape(-1)
    p = np.zeros_like(s)
    _load().orc_precond_norm(C.byref(g), _ptr(s), _ptr(p))
    return p.reshape(img_shape(g))


def rdp_value(g, f, gamma_R, eps):
    return _load().orc_rdp_value(C.byref(g), _ptr(_f64(f).reshape(-1)), gamma_R, eps)


def rdp_grad(g, f, gamma_R, eps):
    f = _f64(f).reshape(-1)
    out = np.zeros_like(f)
    _load().orc_rdp_grad(C.byref(g), _ptr(f), gamma_R, eps, _ptr(out))
    return out.reshape(img_shape(g))


def rdp_hess_apply(g, f, gamma_R, eps, x):
    f = _f64(f).reshape(-1)
    x = _f64(x).reshape(-1)
    out = np.zeros_like(f)
    _load().orc_rdp_hess_apply(C.byref(g), _ptr(f), gamma_R, eps, _ptr(x), _ptr(out))
    return out.reshape(img_shape(g))


def grad_mag(g, f):
    f = _f64(f).reshape(-1)
    out = np.zeros_like(f)
    _load().orc_grad_mag(C.byref(g), _ptr(f), _ptr(out))
    return out.reshape(img_shape(g))


def fidelity(g, f, y, r):
    return _load().orc_fidelity(C.byref(g), _ptr(_f64(f).reshape(-1)),
                                _ptr(_f64(y).reshape(-1)), _ptr(_f64(r).reshape(-1)))


def objective(g, f, y, r, beta, gamma_R, eps):
    return _load().orc_objective(C.byref(g), _ptr(_f64(f).reshape(-1)), _ptr(_f64(y).reshape(-1)),
                                 _ptr(_f64(r).reshape(-1)), beta, gamma_R, eps)


def relax(p, k): return _load().orc_relax(C.byref(p), k)
def nesterov_next(t): return _load().orc_nesterov_next(t)
def km_alpha(p, J): return _load().orc_km_alpha(C.byref(p), J)


def default_U(g, f0, y, r):
    return _load().orc_default_U(C.byref(g), _ptr(_f64(f0).reshape(-1)),
                                 _ptr(_f64(y).reshape(-1)), _ptr(_f64(r).reshape(-1)))


@dataclass
class Recon:
    """Stateful oracle reconstruction: Table I one subiteration at a time."""
    g: _Geom
    p: _Params
    f: np.ndarray
    y: np.ndarray
    r: np.ndarray

    def __post_init__(self):
        self.f = _f64(self.f).reshape(-1).copy()
        self.y = _f64(self.y).reshape(-1)
        self.r = _f64(self.r).reshape(-1)
        self.pnorm = precond_norm(self.g, sensitivity(self.g)).reshape(-1).copy()
        self.frozen = np.zeros_like(self.f)
        self.st = _State()
        _load().orc_state_init(C.byref(self.st))

    def subiteration(self, want_nu=False):
        nu = np.zeros_like(self.f) if want_nu else None
        rc = _load().orc_subiteration(C.byref(self.g), C.byref(self.p), C.byref(self.st),
                                      _ptr(self.f), _ptr(self.y), _ptr(self.r), _ptr(self.pnorm),
                                      _ptr(self.frozen), _ptr(nu))
        if rc != 0:
            raise RuntimeError("oracle subiteration failed")
        return nu

    def clone_with(self, f):
        """Same position, Nesterov t and frozen nu, with iterate f (for one-step
        comparisons from a given input)."""
        c = Recon.__new__(Recon)
        c.g, c.p = self.g, self.p
        c.f = _f64(f).reshape(-1).copy()
        c.y, c.r, c.pnorm = self.y, self.r, self.pnorm
        c.frozen = self.frozen.copy()
        c.st = _State()
        c.st.k, c.st.i, c.st.t_nest, c.st.have_frozen = self.st.k, self.st.i, self.st.t_nest, self.st.have_frozen
        return c

    def image(self):
        return self.f.reshape(img_shape(self.g)).copy()

    def objective(self):
        return objective(self.g, self.f, self.y, self.r, self.p.beta, self.p.gamma_R, self.p.eps)


def reconstruct(g, p, f0, y, r, n_iter, want_obj=True):
    f = _f64(f0).reshape(-1).copy()
    obj = np.zeros(n_iter + 1) if want_obj else None
    rc = _load().orc_reconstruct(C.byref(g), C.byref(p), _ptr(f), _ptr(_f64(y).reshape(-1)),
                                 _ptr(_f64(r).reshape(-1)), n_iter, _ptr(obj))
    if rc != 0:
        raise RuntimeError("oracle reconstruct failed")
    return f.reshape(img_shape(g)), obj
