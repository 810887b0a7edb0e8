"""ctypes binding of libhho.so (C ABI in include/hho.h, include/hho_inspect.h, include/hho_sdirk.h).

Argument marshalling only: every step of the explicit Runge-Kutta path runs in the
HIP kernels of the library.  If the library is not built this module raises; there is
no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhho.so")

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_MESH", 3: "ERR_SINGULAR", 4: "ERR_DEVICE", 5: "ERR_OOM",
          6: "ERR_UNSTABLE"}


class HHOError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class Unstable(HHOError):
    pass


class _Mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("xy", C.c_void_p), ("n_cells", C.c_int32),
                ("cell_ptr", C.c_void_p), ("cell_vtx", C.c_void_p), ("medium", C.c_void_p),
                ("rho", C.c_void_p), ("a", C.c_void_p), ("b", C.c_void_p)]


class _Mesh3d(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("xyz", C.c_void_p), ("n_cells", C.c_int32),
                ("cell_ptr", C.c_void_p), ("cell_vtx", C.c_void_p), ("medium", C.c_void_p),
                ("rho", C.c_void_p), ("a", C.c_void_p), ("b", C.c_void_p)]


class _SdirkParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("mixed", C.c_int32), ("alpha", C.c_int32), ("eta_f", C.c_double),
                ("eta_s", C.c_double), ("stab_speed", C.c_int32), ("ell", C.c_double), ("stages", C.c_int32),
                ("dt", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32), ("device", C.c_int32),
                ("stream", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("rk_stages", C.c_int32), ("eta_f", C.c_double), ("eta_s", C.c_double),
                ("stab_speed", C.c_int32), ("dtype", C.c_int32), ("n_shots", C.c_int32),
                ("record_energy", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p)]


EXPORTS = {
    # name: (restype, argtypes)
    "hho_setup": (C.c_int, [C.POINTER(_Mesh), C.POINTER(_Params), C.POINTER(C.c_void_p)]),
    "hho_setup3d": (C.c_int, [C.POINTER(_Mesh3d), C.POINTER(_Params), C.POINTER(C.c_void_p)]),
    "hho_destroy": (None, [C.c_void_p]),
    "hho_last_error": (C.c_char_p, [C.c_void_p]),
    "hho_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "hho_set_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    "hho_get_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    "hho_set_sources": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32] + [C.c_void_p] * 5),
    "hho_set_ricker_ic": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_int32]),
    "hho_set_loads": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hho_receivers": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "hho_erk_step": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_int32]),
    "hho_reserve_steps": (C.c_int, [C.c_void_p, C.c_int32]),
    "hho_synchronize": (C.c_int, [C.c_void_p]),
    "hho_get_traces": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "hho_energy": (C.c_int, [C.c_void_p, C.c_void_p]),
    "hho_energy_noalloc": (C.c_int, [C.c_void_p, C.c_void_p]),
    "hho_energy_history": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "hho_autotune": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "hho_set_launch": (C.c_int, [C.c_void_p, C.c_int32]),
    "hho_set_tuning": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "hho_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "hho_dt_cfl": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_double)]),
    "hho_set_dt_scale": (C.c_int, [C.c_void_p, C.c_void_p]),
    "hho_cfl_search": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_int32,
                                 C.POINTER(C.c_int32)]),
    "hho_adjoint_step": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_void_p,
                                   C.POINTER(C.c_double), C.c_void_p]),
    "hho_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
    "hho_batch_destroy": (None, [C.c_void_p]),
    "hho_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "hho_batch_erk_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "hho_batch_last_time": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "hho_inspect_create": (C.c_int, [C.POINTER(_Mesh), C.POINTER(_Params), C.POINTER(C.c_void_p)]),
    "hho_inspect3d_create": (C.c_int, [C.POINTER(_Mesh3d), C.POINTER(_Params), C.POINTER(C.c_void_p)]),
    "hho_inspect_destroy": (None, [C.c_void_p]),
    "hho_inspect_sizes": (C.c_int, [C.c_void_p, C.c_void_p]),
    "hho_inspect_arrays": (C.c_int, [C.c_void_p] + [C.c_void_p] * 6),
    "hho_inspect_grad_coefs": (C.c_int, [C.c_void_p, C.c_void_p]),
    "hho_inspect_cell_tables": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "hho_inspect_erk": (C.c_int, [C.c_int32, C.c_void_p]),
    "hho_inspect_dt_cfl": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double)]),
    "hho_sdirk_setup": (C.c_int, [C.POINTER(_Mesh), C.POINTER(_SdirkParams), C.POINTER(C.c_void_p)]),
    "hho_sdirk_destroy": (None, [C.c_void_p]),
    "hho_sdirk_last_error": (C.c_char_p, [C.c_void_p]),
    "hho_sdirk_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "hho_sdirk_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "hho_sdirk_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "hho_sdirk_set_sources": (C.c_int, [C.c_void_p, C.c_int32] + [C.c_void_p] * 5),
    "hho_sdirk_set_ricker_ic": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32]),
    "hho_sdirk_step": (C.c_int, [C.c_void_p, C.c_double, C.c_int32]),
    "hho_sdirk_energy": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "hho_sdirk_receivers": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "hho_sdirk_get_traces": (C.c_int, [C.c_void_p, C.c_void_p]),
    "hho_sdirk_footprint": (C.c_int, [C.c_void_p, C.c_void_p]),
    "hho_sdirk_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "hho_sdirk_inspect_sizes": (C.c_int, [C.POINTER(_Mesh), C.POINTER(_SdirkParams), C.c_void_p]),
    "hho_sdirk_inspect_face_matrix": (C.c_int, [C.POINTER(_Mesh), C.POINTER(_SdirkParams)] + [C.c_void_p] * 4),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhho.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libhho.so is not built (%s): run `python -m paper_2505_15771_amd.build`" % path)
    # PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).  Loading torch
    # first makes libhho.so bind to that runtime, so one HIP runtime serves both and device
    # pointers and streams taken from torch tensors are valid in the library's calls.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _mesh_struct(mesh, keep):
    xy = np.ascontiguousarray(mesh["xy"], np.float64).reshape(-1)
    arrs = dict(xy=xy,
                cell_ptr=np.ascontiguousarray(mesh["cell_ptr"], np.int32),
                cell_vtx=np.ascontiguousarray(mesh["cell_vtx"], np.int32),
                medium=np.ascontiguousarray(mesh["medium"], np.uint8),
                rho=np.ascontiguousarray(mesh["rho"], np.float64),
                a=np.ascontiguousarray(mesh["a"], np.float64),
                b=np.ascontiguousarray(mesh["b"], np.float64))
    keep.update(arrs)
    m = _Mesh()
    m.n_vertices = len(xy) // 2
    m.n_cells = len(arrs["cell_ptr"]) - 1
    for name in ("xy", "cell_ptr", "cell_vtx", "medium", "rho", "a", "b"):
        setattr(m, name, arrs[name].ctypes.data)
    return m


def _mesh3d_struct(mesh, keep):
    """Three-dimensional mesh: xyz [n_vertices, 3] and either cell_ptr / cell_vtx (CSR) or `cells`
    (a list of 4- or 8-tuples of vertex ids)."""
    xyz = np.ascontiguousarray(mesh["xyz"], np.float64).reshape(-1)
    if "cell_ptr" in mesh:
        ptr, vtx = mesh["cell_ptr"], mesh["cell_vtx"]
    else:
        cells = mesh["cells"]
        ptr = np.concatenate([[0], np.cumsum([len(c) for c in cells])])
        vtx = np.concatenate([np.asarray(c) for c in cells])
    arrs = dict(xyz=xyz,
                cell_ptr=np.ascontiguousarray(ptr, np.int32),
                cell_vtx=np.ascontiguousarray(vtx, np.int32),
                medium=np.ascontiguousarray(mesh["medium"], np.uint8),
                rho=np.ascontiguousarray(mesh["rho"], np.float64),
                a=np.ascontiguousarray(mesh["a"], np.float64),
                b=np.ascontiguousarray(mesh["b"], np.float64))
    keep.update(arrs)
    m = _Mesh3d()
    m.n_vertices = len(xyz) // 3
    m.n_cells = len(arrs["cell_ptr"]) - 1
    for name in ("xyz", "cell_ptr", "cell_vtx", "medium", "rho", "a", "b"):
        setattr(m, name, arrs[name].ctypes.data)
    return m


def _params(k, rk_stages, eta_f, eta_s, stab_speed, dtype, n_shots, record_energy, device, stream):
    p = _Params()
    p.k, p.rk_stages, p.eta_f, p.eta_s = int(k), int(rk_stages), float(eta_f), float(eta_s)
    p.stab_speed = int(stab_speed)
    p.dtype = {"f64": 0, "float64": 0, 0: 0, "f32": 1, "float32": 1, 1: 1}[dtype]
    p.n_shots, p.record_energy, p.device = int(n_shots), int(bool(record_energy)), int(device)
    p.stream = stream
    return p


def _check(lib, code, h):
    if code != 0:
        msg = lib.hho_last_error(h).decode()
        raise (Unstable if code == 6 else HHOError)(code, msg)


class Engine:
    """One discretisation on one GPU (hho_setup, or hho_setup3d for a mesh with "xyz"); see
    include/hho.h for the semantics.

    State arrays are float64 in the per-cell layout of hho.h, either numpy arrays
    (host) or contiguous float64 torch cuda tensors (device)."""

    def __init__(self, mesh, k, rk_stages=4, eta_f=0.8, eta_s=1.5, stab_speed=1, dtype="f64", n_shots=1,
                 record_energy=False, device=0, stream=None):
        lib = load_library()
        self.lib = lib
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except Exception:
                stream = None
        self.stream = stream
        keep = {}
        self.dim = 3 if "xyz" in mesh else 2
        m = _mesh3d_struct(mesh, keep) if self.dim == 3 else _mesh_struct(mesh, keep)
        p = _params(k, rk_stages, eta_f, eta_s, stab_speed, dtype, n_shots, record_energy, device, stream)
        h = C.c_void_p()
        setup = lib.hho_setup3d if self.dim == 3 else lib.hho_setup
        _check(lib, setup(C.byref(m), C.byref(p), C.byref(h)), None)
        self._h = h
        self.k, self.n_shots, self.record_energy = k, n_shots, record_energy
        self.medium = keep["medium"].copy()
        nd, nc, nf = C.c_int64(), C.c_int32(), C.c_int32()
        self._call(lib.hho_sizes, C.byref(nd), C.byref(nc), C.byref(nf))
        self.n_dof, self.n_cells, self.n_faces = nd.value, nc.value, nf.value
        self.n_rec = 0
        self.last_steps = 0

    def _call(self, fn, *args):
        _check(self.lib, fn(self._h, *args), self._h)

    def close(self):
        if getattr(self, "_h", None):
            self.lib.hho_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _dev_ptr(t):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            return None
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError("device state must be a contiguous float64 cuda tensor")
        return C.c_void_p(t.data_ptr())

    def set_state(self, U, shot=0):
        try:
            dp = self._dev_ptr(U)
        except ImportError:
            dp = None
        if dp is not None:
            if U.numel() != self.n_dof:
                raise ValueError("state has %d values, expected %d" % (U.numel(), self.n_dof))
            self._call(self.lib.hho_set_state, int(shot), dp, 1)
            return
        U = np.ascontiguousarray(U, np.float64).reshape(-1)
        if U.size != self.n_dof:
            raise ValueError("state has %d values, expected %d" % (U.size, self.n_dof))
        self._call(self.lib.hho_set_state, int(shot), _ptr(U), 0)

    def get_state(self, shot=0, out=None):
        if out is not None:
            dp = self._dev_ptr(out)
            if dp is not None:
                self._call(self.lib.hho_get_state, int(shot), dp, 1)
                return out
        U = np.zeros(self.n_dof)
        self._call(self.lib.hho_get_state, int(shot), _ptr(U), 0)
        return U

    def set_sources(self, shot, xy, direction, f0, t0, amp):
        """Ricker point forces of one shot: positions and directions with `dim` components each."""
        xy = np.ascontiguousarray(np.asarray(xy, np.float64).reshape(-1))
        n = len(xy) // self.dim
        d = np.ascontiguousarray(np.broadcast_to(np.asarray(direction, np.float64), (n, self.dim)).reshape(-1))
        arr = lambda v: np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float64), (n,)))
        f0, t0, amp = arr(f0), arr(t0), arr(amp)
        self._call(self.lib.hho_set_sources, int(shot), n, _ptr(xy), _ptr(d), _ptr(f0), _ptr(t0), _ptr(amp))

    def set_ricker_ic(self, center, lam, theta=1.0, field=1, shot=0):
        """hho_set_ricker_ic: the shot's state becomes the projected field of eq. ricker_ic
        (field 1: velocity, field 0: pressure pulse) centred at `center` with wavelength lam."""
        self._call(self.lib.hho_set_ricker_ic, int(shot), float(center[0]), float(center[1]), float(theta),
                   float(lam), int(field))

    def set_loads(self, g, omega, phase):
        g = np.ascontiguousarray(np.asarray(g, np.float64).reshape(-1))
        om = np.ascontiguousarray(np.atleast_1d(np.asarray(omega, np.float64)))
        ph = np.ascontiguousarray(np.atleast_1d(np.asarray(phase, np.float64)))
        if g.size != len(om) * self.n_dof:
            raise ValueError("load vectors must hold n_terms * n_dof values")
        self._call(self.lib.hho_set_loads, len(om), _ptr(g), _ptr(om), _ptr(ph))

    def set_receivers(self, xy, field):
        xy = np.ascontiguousarray(np.asarray(xy, np.float64).reshape(-1))
        fld = np.ascontiguousarray(np.asarray(field, np.int32).reshape(-1))
        self._call(self.lib.hho_receivers, len(fld), _ptr(xy), _ptr(fld))
        self.n_rec = len(fld)

    def erk_step(self, t0, dt, n_steps):
        self._call(self.lib.hho_erk_step, float(t0), float(dt), int(n_steps))
        self.last_steps = int(n_steps)

    def reserve_steps(self, n_steps):
        """Size the receiver and energy histories for calls of up to n_steps (hho_reserve_steps)."""
        self._call(self.lib.hho_reserve_steps, int(n_steps))

    def adjoint(self, t0, dt, n_steps, d_obs=None, ckpt_every=0):
        """Misfit J and dJ/d(materials) [n_cells, 3] by the discrete adjoint (hho_adjoint_step).

        d_obs: [n_shots, n_steps, n_rec, 2] (or [n_steps, n_rec, 2] for one shot).  Leaves the
        state at U^{n_steps} and the forward traces readable, like erk_step."""
        if self.n_rec:
            d = np.ascontiguousarray(np.asarray(d_obs, np.float64))
            if d.size != self.n_shots * n_steps * self.n_rec * 2:
                raise ValueError("d_obs must hold n_shots * n_steps * n_rec * 2 values")
        else:
            d = None
        J = C.c_double()
        grad = np.zeros((self.n_cells, 3))
        self._call(self.lib.hho_adjoint_step, float(t0), float(dt), int(n_steps), int(ckpt_every), _ptr(d),
                   C.byref(J), _ptr(grad))
        self.last_steps = int(n_steps)
        return J.value, grad

    def synchronize(self):
        self._call(self.lib.hho_synchronize)

    def traces(self, shot=0):
        """[steps, receivers, 2] (two dimensions: p, 0 or v_x, v_y) or [steps, receivers, 3]."""
        out = np.zeros((self.last_steps, self.n_rec, self.dim))
        if self.n_rec and self.last_steps:
            self._call(self.lib.hho_get_traces, int(shot), _ptr(out))
        return out

    def energy(self):
        E = np.zeros(self.n_shots)
        self._call(self.lib.hho_energy, _ptr(E))
        return E

    def energy_noalloc(self, out):
        """hho_energy_noalloc: energies into `out`, a contiguous float64 cuda tensor of n_shots
        values, on the context's stream (no device allocation, no synchronisation)."""
        if not (out.is_cuda and out.is_contiguous() and str(out.dtype) == "torch.float64"
                and out.numel() == self.n_shots):
            raise ValueError("energy_noalloc: out must be a contiguous float64 cuda tensor of n_shots values")
        self._call(self.lib.hho_energy_noalloc, C.c_void_p(out.data_ptr()))

    def autotune(self):
        """Time the stage kernel in every launch shape and store policy, keep the fastest;
        returns its lanes."""
        lanes = C.c_int32()
        self._call(self.lib.hho_autotune, C.byref(lanes))
        return lanes.value

    def set_launch(self, lanes):
        self._call(self.lib.hho_set_launch, int(lanes))

    TUNE_NT_STORES = 1

    def set_tuning(self, lanes, flags):
        """Launch shape by lane count and flags (TUNE_NT_STORES: non-temporal stage stores)."""
        self._call(self.lib.hho_set_tuning, int(lanes), int(flags))

    def tuning(self):
        """(lanes, flags) of the current launch configuration."""
        lanes, flags = C.c_int32(), C.c_int32()
        self._call(self.lib.hho_get_tuning, C.byref(lanes), C.byref(flags))
        return lanes.value, flags.value

    def set_dt_scale(self, scale=None):
        """Per-shot multipliers of dt (None: all 1)."""
        if scale is None:
            self._call(self.lib.hho_set_dt_scale, None)
        else:
            sc = np.ascontiguousarray(scale, dtype=np.float64)
            if sc.shape != (self.n_shots,):
                raise ValueError("one multiplier per shot")
            self._call(self.lib.hho_set_dt_scale, _ptr(sc))

    def cfl_search(self, t_final, n_start, delta=0.01, eps=0.05, max_rounds=100, cap=4096):
        """Algorithm algo_CFL with the shots as simultaneous candidates (hho_cfl_search): returns
        (last stable N, first unstable N, [(N, largest relative energy increase), ...])."""
        ns, nu, cnt = C.c_int32(), C.c_int32(), C.c_int32()
        tried = np.zeros(cap, np.int32)
        growth = np.zeros(cap)
        self._call(self.lib.hho_cfl_search, float(t_final), int(n_start), float(delta), float(eps),
                   int(max_rounds), C.byref(ns), C.byref(nu), _ptr(tried), _ptr(growth), int(cap), C.byref(cnt))
        m = min(cnt.value, cap)
        return ns.value, nu.value, list(zip(tried[:m].tolist(), growth[:m].tolist()))

    def dt_cfl(self, factor=1.0):
        """CFL-limited time step (eq. CFL with the paper's CFL* per cell shape) times factor."""
        dt = C.c_double()
        self._call(self.lib.hho_dt_cfl, float(factor), C.byref(dt))
        return dt.value

    def energy_history(self, shot=0):
        E = np.zeros(max(self.last_steps, 1))
        self._call(self.lib.hho_energy_history, int(shot), _ptr(E))
        return E[:self.last_steps]


def erk_coefficients(stages):
    """Stage-combine coefficients of the stage kernel (hho_inspect_erk): [stages, 9] array of
    c, cY, ck, cb, qa, qb, cd, q_write, q_read."""
    lib = load_library()
    out = np.zeros((stages, 9))
    _check(lib, lib.hho_inspect_erk(int(stages), _ptr(out)), None)
    return out


class Inspect:
    """Host-only view of the execution plan (include/hho_inspect.h)."""

    def __init__(self, mesh, k, eta_f=0.8, eta_s=1.5, stab_speed=1, n_shots=1):
        lib = load_library()
        self.lib = lib
        keep = {}
        self.dim = 3 if "xyz" in mesh else 2
        m = _mesh3d_struct(mesh, keep) if self.dim == 3 else _mesh_struct(mesh, keep)
        p = _params(k, 4, eta_f, eta_s, stab_speed, "f64", n_shots, False, 0, None)
        h = C.c_void_p()
        create = lib.hho_inspect3d_create if self.dim == 3 else lib.hho_inspect_create
        _check(lib, create(C.byref(m), C.byref(p), C.byref(h)), None)
        self._h = h
        sz = np.zeros(10, np.int64)
        lib.hho_inspect_sizes(h, _ptr(sz))
        (self.N, self.F, self.n_ic, self.max_nf, self.n_groups, ntab, self.n_cells, self.n_faces, self.cpb,
         self.n_blocks) = (int(v) for v in sz)
        self.tables = np.zeros(ntab)
        self.groups = np.zeros((self.n_groups, 6), np.int32)
        self.link = np.zeros((self.max_nf, self.n_ic), np.int32)
        self.c0 = np.zeros((self.max_nf, self.n_ic))
        self.mat = np.zeros((6, self.n_ic))
        self.ic_of_cell = np.zeros(self.n_cells, np.int32)
        lib.hho_inspect_arrays(h, _ptr(self.tables), _ptr(self.groups), _ptr(self.link), _ptr(self.c0),
                               _ptr(self.mat), _ptr(self.ic_of_cell))
        self.gm = np.zeros((8, self.n_ic))
        lib.hho_inspect_grad_coefs(h, _ptr(self.gm))
        self.ic_tab = np.zeros(self.n_ic, np.int32)
        self.pooled = np.zeros(self.n_groups, np.int32)
        lib.hho_inspect_cell_tables(h, _ptr(self.ic_tab), _ptr(self.pooled))
        self.dt_cfl = {}
        for s in ((2, 3, 4) if self.dim == 2 else ()):
            dt = C.c_double()
            _check(lib, lib.hho_inspect_dt_cfl(h, s, 1.0, C.byref(dt)), None)
            self.dt_cfl[s] = dt.value
        lib.hho_inspect_destroy(h)
        self._h = None


class Batch:
    """Several engines advanced together from captured graphs (hho_batch_*)."""

    def __init__(self, engines):
        lib = load_library()
        self.lib = lib
        self.engines = list(engines)
        arr = (C.c_void_p * len(self.engines))(*[e._h.value for e in self.engines])
        h = C.c_void_p()
        code = lib.hho_batch_create(arr, len(self.engines), C.byref(h))
        if code != 0:
            raise HHOError(code, lib.hho_last_error(None).decode())
        self._h = h

    def erk_step(self, t0, dt, n_steps):
        n = len(self.engines)
        t0 = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, np.float64), (n,)))
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, np.float64), (n,)))
        code = self.lib.hho_batch_erk_step(self._h, _ptr(t0), _ptr(dt), int(n_steps))
        for e in self.engines:
            e.last_steps = int(n_steps)
        if code != 0:
            msg = self.lib.hho_batch_last_error(self._h).decode()
            raise (Unstable if code == 6 else HHOError)(code, msg)

    def reserve_steps(self, n_steps):
        """hho_reserve_steps on every engine of the batch."""
        for e in self.engines:
            e.reserve_steps(n_steps)

    def last_time_ms(self):
        """Device time of the graph replays of the last erk_step call (HIP events), ms."""
        ms = C.c_double()
        code = self.lib.hho_batch_last_time(self._h, C.byref(ms))
        if code != 0:
            raise HHOError(code, "hho_batch_last_time")
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            self.lib.hho_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _sdirk_params(k, mixed, alpha, eta_f, eta_s, stab_speed, ell, stages, dt, tol, max_iter, device, stream):
    p = _SdirkParams()
    p.k, p.mixed, p.alpha = int(k), int(mixed), int(alpha)
    p.eta_f, p.eta_s, p.stab_speed, p.ell = float(eta_f), float(eta_s), int(stab_speed), float(ell)
    p.stages, p.dt, p.tol, p.max_iter = int(stages), float(dt), float(tol), int(max_iter)
    p.device, p.stream = int(device), stream
    return p


def _sdirk_check(lib, code, h):
    if code != 0:
        msg = lib.hho_sdirk_last_error(h).decode()
        raise (Unstable if code == 6 else HHOError)(code, msg)


class SdirkEngine:
    """SDIRK(stages, stages+1) stepping with static condensation of the cell unknowns and a
    BiCGStab face solve (hho_sdirk_setup); see include/hho_sdirk.h.  State arrays are float64 in
    that header's per-cell layout, numpy (host) or contiguous float64 torch cuda tensors."""

    def __init__(self, mesh, k, dt, stages=3, mixed=True, alpha=1, eta_f=1.0, eta_s=1.0, stab_speed=1, ell=0.0,
                 tol=1e-10, max_iter=2000, device=0, stream=None):
        lib = load_library()
        self.lib = lib
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except Exception:
                stream = None
        keep = {}
        m = _mesh_struct(mesh, keep)
        p = _sdirk_params(k, mixed, alpha, eta_f, eta_s, stab_speed, ell, stages, dt, tol, max_iter, device, stream)
        h = C.c_void_p()
        _sdirk_check(lib, lib.hho_sdirk_setup(C.byref(m), C.byref(p), C.byref(h)), None)
        self._h = h
        self.k, self.dt, self.stages = k, dt, stages
        nd, nf, nnz = C.c_int64(), C.c_int32(), C.c_int64()
        self._call(lib.hho_sdirk_sizes, C.byref(nd), C.byref(nf), C.byref(nnz))
        self.n_dof, self.n_face_dof, self.nnz = nd.value, nf.value, nnz.value

    def _call(self, fn, *args):
        _sdirk_check(self.lib, fn(self._h, *args), self._h)

    def close(self):
        if getattr(self, "_h", None):
            self.lib.hho_sdirk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, U):
        dp = Engine._dev_ptr(U)
        if dp is not None:
            self._call(self.lib.hho_sdirk_set_state, dp, 1)
            return
        U = np.ascontiguousarray(U, np.float64)
        if U.size != self.n_dof:
            raise ValueError("state has %d values, expected %d" % (U.size, self.n_dof))
        self._call(self.lib.hho_sdirk_set_state, _ptr(U), 0)

    def set_ricker_ic(self, center, lam, theta=1.0, field=1):
        """hho_sdirk_set_ricker_ic: the projected field of eq. ricker_ic as the state."""
        self._call(self.lib.hho_sdirk_set_ricker_ic, float(center[0]), float(center[1]), float(theta), float(lam),
                   int(field))

    def get_state(self, out=None):
        if out is not None and Engine._dev_ptr(out) is not None:
            self._call(self.lib.hho_sdirk_get_state, Engine._dev_ptr(out), 1)
            return out
        U = np.zeros(self.n_dof)
        self._call(self.lib.hho_sdirk_get_state, _ptr(U), 0)
        return U

    def set_sources(self, xy, direction, f0, t0, amp):
        xy = np.ascontiguousarray(np.asarray(xy, np.float64).reshape(-1))
        n = len(xy) // 2
        d = np.ascontiguousarray(np.broadcast_to(np.asarray(direction, np.float64), (n, 2)).reshape(-1))
        arr = lambda v: np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float64), (n,)))
        f0, t0, amp = arr(f0), arr(t0), arr(amp)
        self._call(self.lib.hho_sdirk_set_sources, n, _ptr(xy), _ptr(d), _ptr(f0), _ptr(t0), _ptr(amp))

    def set_receivers(self, xy, field):
        xy = np.ascontiguousarray(np.asarray(xy, np.float64).reshape(-1))
        field = np.ascontiguousarray(np.asarray(field, np.int32).reshape(-1))
        self._call(self.lib.hho_sdirk_receivers, len(field), _ptr(xy), _ptr(field))
        self.n_rec = len(field)

    def step(self, t0, n_steps):
        self._call(self.lib.hho_sdirk_step, float(t0), int(n_steps))
        self.last_steps = int(n_steps)

    def traces(self):
        """[n_steps, n_rec, 2] point values after every step of the last step() call."""
        out = np.zeros((self.last_steps, getattr(self, "n_rec", 0), 2))
        if out.size:
            self._call(self.lib.hho_sdirk_get_traces, _ptr(out))
        return out

    def energy(self):
        e = C.c_double()
        self._call(self.lib.hho_sdirk_energy, C.byref(e))
        return e.value

    def footprint(self):
        """dict of the device plan sizes (hho_sdirk_footprint)."""
        sz = np.zeros(7, np.int64)
        self._call(self.lib.hho_sdirk_footprint, _ptr(sz))
        keys = ("n_dof", "n_face_dof", "nnz", "precond_nnz", "cell_matrix_values", "n_slot", "shared_cols")
        return dict(zip(keys, (int(v) for v in sz)))

    def stats(self):
        """(face solves, BiCGStab iterations, largest final relative residual) since setup."""
        a, b, c = C.c_int64(), C.c_int64(), C.c_double()
        self._call(self.lib.hho_sdirk_stats, C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value


def sdirk_face_matrix(mesh, k, dt, stages=3, mixed=True, alpha=1, eta_f=1.0, eta_s=1.0, stab_speed=1, ell=0.0):
    """Host-only: the condensed face matrix of hho_sdirk_setup as (ptr, col, val, face) with
    face[d] = (lower vertex, higher vertex, index in the face block) of face unknown d."""
    lib = load_library()
    keep = {}
    m = _mesh_struct(mesh, keep)
    p = _sdirk_params(k, mixed, alpha, eta_f, eta_s, stab_speed, ell, stages, dt, 1e-10, 1, 0, None)
    sz = np.zeros(5, np.int64)
    _sdirk_check(lib, lib.hho_sdirk_inspect_sizes(C.byref(m), C.byref(p), _ptr(sz)), None)
    nfd, nnz = int(sz[1]), int(sz[2])
    ptr = np.zeros(nfd + 1, np.int32)
    col = np.zeros(max(nnz, 1), np.int32)
    val = np.zeros(max(nnz, 1))
    face = np.zeros((max(nfd, 1), 3), np.int32)
    _sdirk_check(lib, lib.hho_sdirk_inspect_face_matrix(C.byref(m), C.byref(p), _ptr(ptr), _ptr(col), _ptr(val),
                                                        _ptr(face)), None)
    return ptr, col[:nnz], val[:nnz], face[:nfd]
