"""Python binding of the pet_os C ABI (``include/pet_os.h``).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of ``libpet_os.so``.  Tensors are torch CUDA (HIP) float32 contiguous
tensors; pointers and ``torch.cuda.current_stream()`` are passed through.
There is no CPU fallback: without the built library every call raises.

torch is imported before the library is loaded so that both share one HIP
runtime in the process.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpet_os.so")

MODES = {"BSREM": 0, "M1": 1, "M2": 2, "P1": 3, "P2": 4, "OSEM": 5}
ERRORS = {-1: "INVALID_ARG", -2: "OUT_OF_MEMORY", -3: "DEVICE", -4: "BUDGET", -5: "NUMERIC",
          -6: "TIMEOUT", -7: "STATE_MISMATCH"}

# every symbol declared in include/pet_os.h
EXPORTS = ["pet_os_last_error", "pet_os_version", "pet_os_create_geometry", "pet_os_destroy_geometry",
           "pet_os_create_geometry_attenuated", "pet_os_attenuation_factors",
           "pet_os_geometry_info", "pet_os_sensitivity", "pet_os_forward", "pet_os_back",
           "pet_os_objective", "pet_os_default_U", "pet_os_subset_gradient", "pet_os_gradient_angles",
           "pet_os_state_create", "pet_os_state_destroy",
           "pet_os_state_position", "pet_os_subiteration", "pet_os_reconstruct",
           "pet_os_state_export", "pet_os_state_import", "pet_os_run", "pet_os_state_profile",
           "pet_os_state_profile_read", "pet_os_nnz", "pet_os_state_seek", "pet_os_batch_create",
           "pet_os_batch_destroy", "pet_os_batch_add", "pet_os_batch_remove", "pet_os_batch_step",
           "pet_os_batch_run", "pet_os_batch_slot_status", "pet_os_batch_bytes", "pet_os_reconstruct_batch",
           "pet_os_autotune", "pet_os_server_create", "pet_os_server_destroy", "pet_os_submit", "pet_os_wait",
           "pet_os_cancel", "pet_os_server_stats", "pet_os_server_create_simulated", "pet_os_server_inject",
           "pet_os_geometry_shapes", "pet_os_reconstruct_noalloc"]


class PetOSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pet_os error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class GeomDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("vx", C.c_double), ("vy", C.c_double), ("vz", C.c_double),
                ("n_angles", C.c_int32), ("n_radial", C.c_int32), ("ds", C.c_double),
                ("n_rings", C.c_int32), ("max_ring_diff", C.c_int32),
                ("ring_pitch", C.c_double), ("det_radius", C.c_double), ("n_subsets", C.c_int32),
                ("n_subrays", C.c_int32), ("psf_fwhm", C.c_double)]


class Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("beta", C.c_double), ("gamma_R", C.c_double),
                ("eps", C.c_double), ("t_clip", C.c_double), ("U", C.c_double),
                ("lambda0", C.c_double), ("a", C.c_double), ("rho", C.c_double),
                ("delta1", C.c_double), ("delta2", C.c_double), ("nu1", C.c_double),
                ("nu2", C.c_double), ("J0", C.c_int64), ("J1", C.c_int64),
                ("objective_every", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("desc", GeomDesc), ("params", Params), ("f", C.c_void_p), ("y", C.c_void_p), ("r", C.c_void_p),
                ("n_iter", C.c_int32), ("want_objective", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("pad", C.c_int32), ("objective", C.c_double), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_start", C.c_double), ("t_finish", C.c_double),
                ("subiterations", C.c_int64), ("message", C.c_char * 128)]


class ServerStats(C.Structure):
    _fields_ = [("queued", C.c_int64), ("active", C.c_int64), ("ticks", C.c_int64), ("max_active", C.c_int64),
                ("bytes_in_use", C.c_size_t), ("geometries_cached", C.c_int64)]


INJECT = {"admit_oom": 1, "step_failure": 2, "nan_objective": 3, "bad_data": 4}

_lib = None
_P = C.c_void_p


def lib():
    """Load libpet_os.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2111_07886_amd/build.py")
        L = C.CDLL(LIB_PATH)
        i32, i64 = C.c_int32, C.c_int64
        sig = {
            "pet_os_last_error": (C.c_char_p, []),
            "pet_os_version": (C.c_char_p, []),
            "pet_os_create_geometry": (C.c_int, [C.POINTER(GeomDesc), C.POINTER(_P)]),
            "pet_os_create_geometry_attenuated": (C.c_int, [C.POINTER(GeomDesc), _P, C.POINTER(_P)]),
            "pet_os_attenuation_factors": (C.c_int, [_P, _P, _P, _P]),
            "pet_os_destroy_geometry": (C.c_int, [_P]),
            "pet_os_geometry_info": (C.c_int, [_P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)]),
            "pet_os_sensitivity": (C.c_int, [_P, _P, _P]),
            "pet_os_forward": (C.c_int, [_P, _P, i32, _P, _P]),
            "pet_os_back": (C.c_int, [_P, _P, i32, _P, _P]),
            "pet_os_objective": (C.c_int, [_P, C.POINTER(Params), _P, _P, _P, C.POINTER(C.c_double), _P]),
            "pet_os_default_U": (C.c_int, [_P, _P, _P, _P, C.POINTER(C.c_double), _P]),
            "pet_os_subset_gradient": (C.c_int, [_P, C.POINTER(Params), _P, _P, _P, i32, _P, _P]),
            "pet_os_gradient_angles": (C.c_int, [_P, _P, _P, _P, C.c_double, C.c_double,
                                                 C.POINTER(C.c_double), C.POINTER(i64), _P]),
            "pet_os_state_create": (C.c_int, [_P, C.POINTER(Params), C.POINTER(_P)]),
            "pet_os_state_destroy": (C.c_int, [_P]),
            "pet_os_state_position": (C.c_int, [_P, C.POINTER(i64), C.POINTER(i32)]),
            "pet_os_subiteration": (C.c_int, [_P, _P, _P, _P, _P]),
            "pet_os_reconstruct": (C.c_int, [_P, C.POINTER(Params), _P, _P, _P, i32,
                                             C.POINTER(C.c_double), _P]),
            "pet_os_reconstruct_noalloc": (C.c_int, [_P, C.POINTER(Params), _P, _P, _P, i32, _P]),
            "pet_os_state_export": (C.c_int, [_P, _P, C.POINTER(C.c_size_t)]),
            "pet_os_state_import": (C.c_int, [_P, _P, C.c_size_t]),
            "pet_os_run": (C.c_int, [_P, _P, _P, _P, i32, C.POINTER(C.c_double), _P]),
            "pet_os_state_profile": (C.c_int, [_P, i32]),
            "pet_os_state_profile_read": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(i64)]),
            "pet_os_nnz": (C.c_int, [_P, i32, C.POINTER(i64)]),
            "pet_os_state_seek": (C.c_int, [_P, i64, i32, C.c_double, _P]),
            "pet_os_batch_create": (C.c_int, [i32, C.POINTER(_P)]),
            "pet_os_batch_destroy": (C.c_int, [_P]),
            "pet_os_batch_add": (C.c_int, [_P, _P, C.POINTER(Params), _P, _P, _P, i32, _P, C.POINTER(i32)]),
            "pet_os_batch_remove": (C.c_int, [_P, i32, _P]),
            "pet_os_batch_step": (C.c_int, [_P, i32, _P]),
            "pet_os_batch_run": (C.c_int, [_P, _P]),
            "pet_os_batch_slot_status": (C.c_int, [_P, i32, C.POINTER(i32), C.POINTER(i64)]),
            "pet_os_batch_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
            "pet_os_reconstruct_batch": (C.c_int, [i32, C.POINTER(_P), C.POINTER(Params), C.POINTER(_P),
                                                   C.POINTER(_P), C.POINTER(_P), C.POINTER(i32), _P]),
            "pet_os_autotune": (C.c_int, [_P, i32, _P]),
            "pet_os_geometry_shapes": (C.c_int, [_P, C.POINTER(i32), C.POINTER(i32)]),
            "pet_os_server_create": (C.c_int, [C.c_size_t, i32, C.POINTER(_P)]),
            "pet_os_server_destroy": (C.c_int, [_P]),
            "pet_os_submit": (C.c_int, [_P, C.POINTER(Request), C.POINTER(C.c_uint64)]),
            "pet_os_wait": (C.c_int, [_P, C.c_uint64, i64, C.POINTER(Result)]),
            "pet_os_cancel": (C.c_int, [_P, C.c_uint64]),
            "pet_os_server_stats": (C.c_int, [_P, C.POINTER(ServerStats)]),
            "pet_os_server_create_simulated": (C.c_int, [C.c_size_t, i32, i64, C.POINTER(_P)]),
            "pet_os_server_inject": (C.c_int, [_P, i32, i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().pet_os_last_error().decode()


def _check(rc):
    if rc != 0:
        raise PetOSError(rc, last_error())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, n: int | None = None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return C.c_void_p(t.data_ptr())


def desc_struct(d: dict) -> GeomDesc:
    g = GeomDesc()
    g.dim = int(d["dim"])
    g.nx, g.ny, g.nz = int(d["nx"]), int(d["ny"]), int(d.get("nz", 1))
    g.vx, g.vy, g.vz = float(d["vx"]), float(d["vy"]), float(d.get("vz", 1.0))
    g.n_angles, g.n_radial, g.ds = int(d["n_angles"]), int(d["n_radial"]), float(d["ds"])
    g.n_rings, g.max_ring_diff = int(d.get("n_rings", 1)), int(d.get("max_ring_diff", 0))
    g.ring_pitch, g.det_radius = float(d.get("ring_pitch", 1.0)), float(d.get("det_radius", 0.0))
    g.n_subsets = int(d["n_subsets"])
    g.n_subrays = int(d.get("n_subrays", 1))
    g.psf_fwhm = float(d.get("psf_fwhm", 0.0))
    return g


def params_struct(p: dict) -> Params:
    q = Params()
    q.mode = MODES[p["mode"]] if isinstance(p["mode"], str) else int(p["mode"])
    osem = q.mode == MODES["OSEM"]
    for k in ("beta", "gamma_R", "eps", "t_clip", "U", "lambda0", "a", "rho", "delta1", "delta2",
              "nu1", "nu2"):
        # OSEM reads only beta, gamma_R and eps (objective); the rest may be absent
        setattr(q, k, float(p.get(k, 0.0) if osem else p[k]))
    q.J0, q.J1 = (int(p.get("J0", 0)), int(p.get("J1", 0))) if osem else (int(p["J0"]), int(p["J1"]))
    q.objective_every = int(p.get("objective_every", 1))
    return q


class Geometry:
    """Handle of pet_os_create_geometry (sensitivity and p computed on creation).
    ``att``: optional per-bin attenuation factors (host array of n_bins
    values), for pet_os_create_geometry_attenuated."""

    def __init__(self, desc: dict, att=None):
        self.desc = dict(desc)
        self._d = desc_struct(desc)
        h = _P()
        if att is None:
            _check(lib().pet_os_create_geometry(C.byref(self._d), C.byref(h)))
        else:
            import numpy as np
            a = np.ascontiguousarray(np.asarray(att, dtype=np.float32).reshape(-1))
            _check(lib().pet_os_create_geometry_attenuated(C.byref(self._d), C.c_void_p(a.ctypes.data),
                                                           C.byref(h)))
        self.handle = h
        nv, nb, npl = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().pet_os_geometry_info(h, C.byref(nv), C.byref(nb), C.byref(npl)))
        self.n_voxels, self.n_bins, self.n_planes = nv.value, nb.value, npl.value

    @property
    def img_shape(self):
        d = self.desc
        return (d["nz"], d["ny"], d["nx"]) if d["dim"] == 3 else (d["ny"], d["nx"])

    @property
    def sino_shape(self):
        return (self.n_planes, self.desc["n_angles"], self.desc["n_radial"])

    def close(self):
        if getattr(self, "handle", None):
            lib().pet_os_destroy_geometry(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sensitivity(self, stream=None):
        out = torch.empty(self.img_shape, device="cuda", dtype=torch.float32)
        _check(lib().pet_os_sensitivity(self.handle, _dev(out), _stream(stream)))
        return out

    def forward(self, f, subset=0, out=None, stream=None):
        if out is None:
            out = torch.zeros(self.sino_shape, device="cuda", dtype=torch.float32)
        _check(lib().pet_os_forward(self.handle, _dev(f, self.n_voxels, "f"), int(subset),
                                    _dev(out, self.n_bins, "q"), _stream(stream)))
        return out

    def back(self, w, subset=0, out=None, stream=None):
        if out is None:
            out = torch.empty(self.img_shape, device="cuda", dtype=torch.float32)
        _check(lib().pet_os_back(self.handle, _dev(w, self.n_bins, "w"), int(subset),
                                 _dev(out, self.n_voxels, "out"), _stream(stream)))
        return out

    def objective(self, params: dict, f, y, r, stream=None) -> float:
        p = params_struct(params)
        phi = C.c_double()
        _check(lib().pet_os_objective(self.handle, C.byref(p), _dev(f, self.n_voxels, "f"),
                                      _dev(y, self.n_bins, "y"), _dev(r, self.n_bins, "r"),
                                      C.byref(phi), _stream(stream)))
        return phi.value

    def subset_gradient(self, params: dict, f, y, r, subset, out=None, stream=None):
        """pet_os_subset_gradient: grad Phi_i(f) (subset 1..M) or grad Phi(f) (0)."""
        if out is None:
            out = torch.empty(self.img_shape, device="cuda", dtype=torch.float32)
        p = params_struct(params)
        _check(lib().pet_os_subset_gradient(self.handle, C.byref(p), _dev(f, self.n_voxels, "f"),
                                            _dev(y, self.n_bins, "y"), _dev(r, self.n_bins, "r"), int(subset),
                                            _dev(out, self.n_voxels, "grad"), _stream(stream)))
        return out

    def gradient_angles(self, h_prev, h_cur, f, smooth_frac=0.01, var_frac=0.2, stream=None):
        """pet_os_gradient_angles: (theta_smooth, theta_variable) in radians and
        the sizes of the two areas."""
        th = (C.c_double * 2)()
        cnt = (C.c_int64 * 2)()
        _check(lib().pet_os_gradient_angles(self.handle, _dev(h_prev, self.n_voxels, "h_prev"),
                                            _dev(h_cur, self.n_voxels, "h_cur"), _dev(f, self.n_voxels, "f"),
                                            float(smooth_frac), float(var_frac), th, cnt, _stream(stream)))
        return th[0], th[1], cnt[0], cnt[1]

    def attenuation_factors(self, mu, out=None, stream=None):
        """pet_os_attenuation_factors: exp(-line integrals of mu) per bin."""
        if out is None:
            out = torch.empty(self.sino_shape, device="cuda", dtype=torch.float32)
        _check(lib().pet_os_attenuation_factors(self.handle, _dev(mu, self.n_voxels, "mu"),
                                                _dev(out, self.n_bins, "att"), _stream(stream)))
        return out

    def shapes(self) -> dict:
        """pet_os_geometry_shapes: {"current": ..., "default": ...}, each
        {"fp_seg", "bp_kind", "bp3_zb", "bp3_dpg"}."""
        cur, dft = (C.c_int32 * 4)(), (C.c_int32 * 4)()
        _check(lib().pet_os_geometry_shapes(self.handle, cur, dft))
        keys = ("fp_seg", "bp_kind", "bp3_zb", "bp3_dpg")
        return {"current": dict(zip(keys, list(cur))), "default": dict(zip(keys, list(dft)))}

    def nnz(self, subset=0) -> int:
        n = C.c_int64()
        _check(lib().pet_os_nnz(self.handle, int(subset), C.byref(n)))
        return n.value

    def default_U(self, f0, y, r, stream=None) -> float:
        U = C.c_double()
        _check(lib().pet_os_default_U(self.handle, _dev(f0, self.n_voxels, "f0"), _dev(y, self.n_bins, "y"),
                                      _dev(r, self.n_bins, "r"), C.byref(U), _stream(stream)))
        return U.value


class State:
    """Handle of pet_os_state_create: one reconstruction advanced subiteration by subiteration."""

    def __init__(self, geom: Geometry, params: dict):
        self.geom = geom
        self._p = params_struct(params)
        h = _P()
        _check(lib().pet_os_state_create(geom.handle, C.byref(self._p), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().pet_os_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def subiteration(self, f, y, r, stream=None):
        g = self.geom
        _check(lib().pet_os_subiteration(self.handle, _dev(f, g.n_voxels, "f"), _dev(y, g.n_bins, "y"),
                                         _dev(r, g.n_bins, "r"), _stream(stream)))

    def run(self, f, y, r, n_iter, want_objective=False, stream=None):
        """pet_os_run: n_iter iterations from the current position; returns the
        objective after each iteration (NaN where not evaluated) or None."""
        g = self.geom
        obj = (C.c_double * max(1, n_iter))() if want_objective else None
        _check(lib().pet_os_run(self.handle, _dev(f, g.n_voxels, "f"), _dev(y, g.n_bins, "y"),
                                _dev(r, g.n_bins, "r"), int(n_iter), obj, _stream(stream)))
        return list(obj)[:n_iter] if want_objective else None

    def seek(self, k: int, i: int, t_nest: float = 1.0, nu_frozen=None):
        """pet_os_state_seek: continue from subiteration (k, i) with Nesterov t
        and (optionally) the frozen nu."""
        nu = None if nu_frozen is None else _dev(nu_frozen, self.geom.n_voxels, "nu_frozen")
        _check(lib().pet_os_state_seek(self.handle, int(k), int(i), float(t_nest), nu))

    def profile(self, kernel: int):
        """Bracket every launch of kernel 0 (forward+ratio), 1 (back+stencil) or
        2 (update) with HIP events; -1 switches off."""
        _check(lib().pet_os_state_profile(self.handle, int(kernel)))

    def profile_read(self):
        ms, n = C.c_double(), C.c_int64()
        _check(lib().pet_os_state_profile_read(self.handle, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def position(self):
        k, i = C.c_int64(), C.c_int32()
        _check(lib().pet_os_state_position(self.handle, C.byref(k), C.byref(i)))
        return k.value, i.value

    def export(self) -> bytes:
        n = C.c_size_t()
        _check(lib().pet_os_state_export(self.handle, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().pet_os_state_export(self.handle, buf, C.byref(n)))
        return buf.raw[: n.value]

    def import_(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().pet_os_state_import(self.handle, buf, len(blob)))


def osem_params(beta=0.0, gamma_R=2.0, eps=1e-12):
    """Parameters of the OSEM initialisation (Sec. IV-C): beta, gamma_R and
    eps only enter the objective evaluations."""
    return dict(mode="OSEM", beta=beta, gamma_R=gamma_R, eps=eps)


def reconstruct_osem_init(geom: Geometry, params: dict, f, y, r, n_osem: int, n_iter: int, stream=None):
    """The clinical procedure of Sec. IV-C: n_osem OSEM iterations on f (in
    place) with the geometry's subsets, then n_iter SDP-BSREM iterations of
    ``params`` from that image (k starts at 0)."""
    st = State(geom, osem_params(params.get("beta", 0.0), params.get("gamma_R", 2.0), params.get("eps", 1e-12)))
    try:
        st.run(f, y, r, n_osem, stream=stream)
    finally:
        st.close()
    return reconstruct(geom, params, f, y, r, n_iter, stream=stream)


def reconstruct(geom: Geometry, params: dict, f, y, r, n_iter: int, want_objective=False, stream=None):
    """pet_os_reconstruct: n_iter iterations in place on f; returns the objective
    trace (list of n_iter+1 floats, NaN where not evaluated) or None."""
    p = params_struct(params)
    obj = (C.c_double * (n_iter + 1))() if want_objective else None
    _check(lib().pet_os_reconstruct(geom.handle, C.byref(p), _dev(f, geom.n_voxels, "f"),
                                    _dev(y, geom.n_bins, "y"), _dev(r, geom.n_bins, "r"), int(n_iter),
                                    obj, _stream(stream)))
    return list(obj) if want_objective else None


NOALLOC_SCRATCH_BYTES = 64 << 20      # PET_OS_NOALLOC_SCRATCH_BYTES


def reconstruct_noalloc(geom: Geometry, params: dict, f, y, r, n_iter: int, stream=None):
    """pet_os_reconstruct_noalloc: pet_os_reconstruct without objectives, with
    the request's scratch in the library's static device array (no device
    allocation); n_iter iterations in place on f."""
    p = params_struct(params)
    _check(lib().pet_os_reconstruct_noalloc(geom.handle, C.byref(p), _dev(f, geom.n_voxels, "f"),
                                            _dev(y, geom.n_bins, "y"), _dev(r, geom.n_bins, "r"), int(n_iter),
                                            _stream(stream)))


class Batch:
    """pet_os_batch: independent reconstructions advanced together, one
    captured batched subiteration per step."""

    def __init__(self, max_slots: int):
        h = _P()
        _check(lib().pet_os_batch_create(int(max_slots), C.byref(h)))
        self.handle = h
        self._keep = {}

    def close(self):
        if getattr(self, "handle", None):
            lib().pet_os_batch_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, geom: Geometry, params: dict, f, y, r, n_iter: int, stream=None) -> int:
        p = params_struct(params)
        slot = C.c_int32()
        _check(lib().pet_os_batch_add(self.handle, geom.handle, C.byref(p), _dev(f, geom.n_voxels, "f"),
                                      _dev(y, geom.n_bins, "y"), _dev(r, geom.n_bins, "r"), int(n_iter),
                                      _stream(stream), C.byref(slot)))
        self._keep[slot.value] = (geom, f, y, r)
        return slot.value

    def remove(self, slot: int, stream=None):
        _check(lib().pet_os_batch_remove(self.handle, int(slot), _stream(stream)))
        self._keep.pop(slot, None)

    def step(self, n_steps: int = 1, stream=None):
        _check(lib().pet_os_batch_step(self.handle, int(n_steps), _stream(stream)))

    def run(self, stream=None):
        _check(lib().pet_os_batch_run(self.handle, _stream(stream)))

    def status(self, slot: int):
        a, rem = C.c_int32(), C.c_int64()
        _check(lib().pet_os_batch_slot_status(self.handle, int(slot), C.byref(a), C.byref(rem)))
        return bool(a.value), rem.value

    def bytes(self) -> int:
        n = C.c_size_t()
        _check(lib().pet_os_batch_bytes(self.handle, C.byref(n)))
        return n.value


def reconstruct_batch(geoms, params, fs, ys, rs, n_iters, stream=None):
    """pet_os_reconstruct_batch: every request in one batch; blocks until done."""
    n = len(geoms)
    G = (_P * n)(*[g.handle for g in geoms])
    P = (Params * n)(*[params_struct(p) for p in params])
    F = (_P * n)(*[_dev(f, g.n_voxels, "f") for f, g in zip(fs, geoms)])
    Y = (_P * n)(*[_dev(y, g.n_bins, "y") for y, g in zip(ys, geoms)])
    R = (_P * n)(*[_dev(r, g.n_bins, "r") for r, g in zip(rs, geoms)])
    N = (C.c_int32 * n)(*[int(k) for k in n_iters])
    _check(lib().pet_os_reconstruct_batch(n, G, P, F, Y, R, N, _stream(stream)))


def autotune(geom: Geometry, force=False, stream=None):
    """pet_os_autotune: pick the projector shapes for this geometry by timing."""
    _check(lib().pet_os_autotune(geom.handle, 1 if force else 0, _stream(stream)))


class Server:
    """pet_os_server: continuous-batching reconstruction server.  With
    simulate=True no device call is made (host scheduling tests)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int, simulate=False, step_us=50):
        h = _P()
        if simulate:
            _check(lib().pet_os_server_create_simulated(int(hbm_budget_bytes), int(max_slots), int(step_us),
                                                        C.byref(h)))
        else:
            _check(lib().pet_os_server_create(int(hbm_budget_bytes), int(max_slots), C.byref(h)))
        self.handle = h
        self.simulate = simulate
        self._keep = {}

    def close(self):
        if getattr(self, "handle", None):
            lib().pet_os_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, desc: dict, params: dict, f=None, y=None, r=None, n_iter=1, want_objective=False) -> int:
        rq = Request()
        rq.desc = desc_struct(desc)
        rq.params = params_struct(params)
        if not self.simulate:
            rq.f = _dev(f, name="f").value
            rq.y = _dev(y, name="y").value
            rq.r = _dev(r, name="r").value
        rq.n_iter = int(n_iter)
        rq.want_objective = 1 if want_objective else 0
        t = C.c_uint64()
        _check(lib().pet_os_submit(self.handle, C.byref(rq), C.byref(t)))
        self._keep[t.value] = (f, y, r)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> dict:
        res = Result()
        _check(lib().pet_os_wait(self.handle, int(ticket), int(timeout_us), C.byref(res)))
        self._keep.pop(ticket, None)
        return dict(status=res.status, objective=res.objective, t_submit=res.t_submit, t_admit=res.t_admit,
                    t_start=res.t_start, t_finish=res.t_finish, subiterations=res.subiterations,
                    message=res.message.decode(errors="replace"))

    def cancel(self, ticket: int):
        _check(lib().pet_os_cancel(self.handle, int(ticket)))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().pet_os_server_stats(self.handle, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def inject(self, kind: str, count: int = 1):
        _check(lib().pet_os_server_inject(self.handle, INJECT[kind], int(count)))
