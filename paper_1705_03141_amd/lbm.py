"""Python binding of the C ABI in ``include/lbm.h`` (argument marshalling only).

Every step of the method runs in the HIP library ``liblbm.so``; this module converts numpy
arrays and problem descriptions into the ABI's plain pointers and sizes.  The functions
``lbm_create``, ``lbm_init_fields``, ``lbm_step`` ... carry the names of the C entry points;
:class:`Lattice` bundles them for one context.  There is no fallback: if the library is
missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lbm.h")
Q = 27

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = range(6)
STATUS_NAMES = {0: "LBM_OK", 1: "LBM_EINVAL", 2: "LBM_ENOMEM", 3: "LBM_EDEVICE", 4: "LBM_EUNSTABLE", 5: "LBM_ESTATE"}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
FIELDS = {"rho_r": 0, "rho_b": 1, "ux": 2, "uy": 3, "uz": 4, "phi": 5, "p": 6}


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("rho_r0", ctypes.c_double), ("rho_b0", ctypes.c_double),
        ("nu_r", ctypes.c_double), ("nu_b", ctypes.c_double),
        ("A", ctypes.c_double), ("beta", ctypes.c_double),
        ("s", ctypes.c_double * Q),
        ("face", ctypes.c_int * 6),
        ("force", ctypes.c_int),
        ("g", ctypes.c_double * 3),
        ("rho_ref", ctypes.c_double),
        ("storage", ctypes.c_int),
    ]


class lbm_diag(ctypes.Structure):
    _fields_ = [("mass_r", ctypes.c_double), ("mass_b", ctypes.c_double), ("umax", ctypes.c_double),
                ("p_in", ctypes.c_double), ("p_out", ctypes.c_double), ("n_in", ctypes.c_longlong),
                ("n_out", ctypes.c_longlong), ("nan_cells", ctypes.c_longlong), ("step", ctypes.c_longlong)]


_D = ctypes.POINTER(ctypes.c_double)
_lib = None


def library():
    """Load ``liblbm.so`` (building it first if it is absent or older than its sources)."""
    global _lib
    if _lib is None:
        from . import build as _build
        if _build.stale():
            _build.build()
        # torch ships its own HIP runtime under the same library name as the system's; loading
        # it first makes the process use one runtime for both (the second one loaded would
        # otherwise resolve to the first and find no GPU)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(lbm_params)
        vp = ctypes.c_void_p
        L.lbm_create.argtypes = [P, vp, ctypes.POINTER(vp)]
        L.lbm_init_fields.argtypes = [vp, _D, _D, _D]
        L.lbm_set_inflow.argtypes = [vp] + [ctypes.c_double] * 5 + [ctypes.c_ulonglong]
        L.lbm_set_tiling.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.lbm_autotune.argtypes = [vp, ctypes.c_int]
        L.lbm_get_tiling.argtypes = [vp] + [ctypes.POINTER(ctypes.c_int)] * 3
        L.lbm_step.argtypes = [vp, ctypes.c_int]
        L.lbm_sync.argtypes = [vp]
        L.lbm_step_count.argtypes = [vp]
        L.lbm_step_count.restype = ctypes.c_longlong
        L.lbm_read_field.argtypes = [vp, ctypes.c_int, _D]
        L.lbm_read_field_box.argtypes = [vp, ctypes.c_int] + [ctypes.c_int] * 6 + [_D]
        L.lbm_read_field_box_noalloc.argtypes = [vp, ctypes.c_int] + [ctypes.c_int] * 6 + [_D]
        L.lbm_read_field_box_noalloc.restype = ctypes.c_int
        L.lbm_coarse_state.argtypes = [vp, ctypes.c_int, ctypes.c_double, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.lbm_coarse_state.restype = ctypes.c_int
        L.lbm_read_populations.argtypes = [vp, _D]
        L.lbm_state_bytes.argtypes = [vp]
        L.lbm_state_bytes.restype = ctypes.c_size_t
        L.lbm_save_state.argtypes = [vp, vp, ctypes.c_size_t]
        L.lbm_load_state.argtypes = [vp, vp, ctypes.c_size_t]
        L.lbm_diagnostics.argtypes = [vp] + [ctypes.c_double] * 5 + [ctypes.POINTER(lbm_diag)]
        L.lbm_last_step_kernel_ms.argtypes = [vp]
        L.lbm_last_step_kernel_ms.restype = ctypes.c_double
        L.lbm_last_error.argtypes = [vp]
        L.lbm_last_error.restype = ctypes.c_char_p
        L.lbm_destroy.argtypes = [vp]
        L.lbm_destroy.restype = None
        L.lbm_selftest_collide_host.argtypes = [P, _D, _D, _D, _D, _D, _D]
        L.lbm_selftest_tile_sets_host.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        for name in ("lbm_sigma_from_A", "lbm_A_from_sigma"):
            getattr(L, name).argtypes = [ctypes.c_double, ctypes.c_double]
            getattr(L, name).restype = ctypes.c_double
        L.lbm_batch_create.argtypes = [P, ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.lbm_batch_case.argtypes = [vp, ctypes.c_int]
        L.lbm_batch_case.restype = vp
        L.lbm_batch_size.argtypes = [vp]
        L.lbm_batch_autotune.argtypes = [vp, ctypes.c_int]
        L.lbm_batch_step.argtypes = [vp, ctypes.c_int]
        L.lbm_batch_sync.argtypes = [vp]
        L.lbm_batch_unstable_cases.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.lbm_batch_unstable_cases.restype = ctypes.c_int
        L.lbm_batch_last_step_ms.argtypes = [vp]
        L.lbm_batch_last_step_ms.restype = ctypes.c_double
        L.lbm_batch_last_error.argtypes = [vp]
        L.lbm_batch_last_error.restype = ctypes.c_char_p
        L.lbm_batch_destroy.argtypes = [vp]
        L.lbm_batch_destroy.restype = None
        for name in header_functions():
            getattr(L, name).restype = getattr(L, name).restype  # resolves every declared symbol
        for name in ("lbm_create", "lbm_init_fields", "lbm_set_inflow", "lbm_set_tiling", "lbm_autotune", "lbm_get_tiling", "lbm_step", "lbm_sync",
                     "lbm_read_field", "lbm_read_field_box", "lbm_read_populations", "lbm_save_state",
                     "lbm_load_state", "lbm_diagnostics", "lbm_selftest_collide_host", "lbm_selftest_tile_sets_host",
                     "lbm_batch_create",
                     "lbm_batch_autotune", "lbm_batch_step", "lbm_batch_sync", "lbm_batch_size"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/lbm.h."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:[a-z_]+\s+)+\**\s*(lbm_[A-Za-z_0-9]+)\s*\(", text, re.M)))


def _ptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _arr(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64)).reshape(-1)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _check(ctx, status):
    if status != LBM_OK:
        msg = library().lbm_last_error(ctx)
        raise LbmError(status, msg.decode() if msg else "")


# ---------------------------------------------------------------- C names

def params_from_problem(pb, storage: str = "f32") -> lbm_params:
    p = lbm_params()
    p.nx, p.ny, p.nz = pb.nx, pb.ny, pb.nz
    p.rho_r0, p.rho_b0, p.nu_r, p.nu_b = pb.rho_r0, pb.rho_b0, pb.nu_r, pb.nu_b
    # a problem may give the interfacial tension instead of A: Eq. (sigma) at the continuous
    # (blue) phase's relaxation time, converted by the library (lbm_A_from_sigma)
    p.A = pb.A if pb.A is not None else A_from_sigma(pb.sigma, pb.nu_b)
    p.beta = pb.beta
    if pb.s is not None:
        for j in range(Q):
            p.s[j] = pb.s[j]
    for k in range(6):
        p.face[k] = int(pb.faces[k])
    p.force = int(pb.force_model)
    for a in range(3):
        p.g[a] = pb.g[a]
    p.rho_ref = pb.rho_ref
    p.storage = STORAGE[storage]
    return p


def lbm_create(params: lbm_params, stream: Optional[int] = None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    st = library().lbm_create(ctypes.byref(params), ctypes.c_void_p(stream) if stream else None, ctypes.byref(ctx))
    _check(None, st)
    return ctx


def lbm_init_fields(ctx, rho_r, rho_b, u=None, n=None):
    rr, rb = _arr(rho_r, n), _arr(rho_b, n)
    uu = _arr(u, 3 * n) if u is not None else None
    _check(ctx, library().lbm_init_fields(ctx, _ptr(rr), _ptr(rb), _ptr(uu)))


def lbm_set_inflow(ctx, xc, yc, diameter, u_normal, noise_rel, seed):
    _check(ctx, library().lbm_set_inflow(ctx, xc, yc, diameter, u_normal, noise_rel, int(seed)))


def lbm_set_tiling(ctx, tx, ty, zchunk):
    _check(ctx, library().lbm_set_tiling(ctx, tx, ty, zchunk))


def lbm_step(ctx, nsteps: int):
    _check(ctx, library().lbm_step(ctx, int(nsteps)))


def lbm_sync(ctx):
    _check(ctx, library().lbm_sync(ctx))


def lbm_destroy(ctx):
    library().lbm_destroy(ctx)


# ---------------------------------------------------------------- convenience class

class Lattice:
    """One lattice on the GPU, built from a :class:`workloads.Problem`."""

    def __init__(self, problem, storage: str = "f32", stream: Optional[int] = None, init: bool = True,
                 tiling: Optional[tuple] = None, _ctx=None):
        self.pb = problem
        self.storage = storage
        self.params = params_from_problem(problem, storage)
        self._owned = _ctx is None
        self.ctx = lbm_create(self.params, stream) if _ctx is None else _ctx
        self.shape = (problem.nz, problem.ny, problem.nx)
        self.n = problem.ncells
        if problem.inflow:
            lbm_set_inflow(self.ctx, problem.xc, problem.yc, problem.diameter, problem.u_in, problem.noise_rel,
                           problem.seed)
        if tiling is not None:
            lbm_set_tiling(self.ctx, *tiling)
        if init:
            self.init_fields(problem.rho_r, problem.rho_b, problem.u)

    def autotune(self, trial_steps: int = 20):
        """Time the supported tile shapes on a scratch lattice and keep the fastest
        (lbm_autotune)."""
        _check(self.ctx, library().lbm_autotune(self.ctx, int(trial_steps)))

    def tiling(self) -> tuple:
        """(tx, ty, zchunk) of the step kernel (lbm_get_tiling)."""
        v = [ctypes.c_int() for _ in range(3)]
        _check(self.ctx, library().lbm_get_tiling(self.ctx, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def close(self):
        if getattr(self, "ctx", None):
            if self._owned:
                lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, rho_r, rho_b, u=None):
        lbm_init_fields(self.ctx, rho_r, rho_b, u, self.n)

    def step(self, n: int = 1):
        lbm_step(self.ctx, n)

    def sync(self):
        lbm_sync(self.ctx)

    @property
    def steps_done(self) -> int:
        return int(library().lbm_step_count(self.ctx))

    def field(self, name: str) -> np.ndarray:
        out = np.empty(self.n)
        _check(self.ctx, library().lbm_read_field(self.ctx, FIELDS[name], _ptr(out)))
        return out.reshape(self.shape)

    def field_box(self, name: str, x0, y0, z0, wx, wy, wz) -> np.ndarray:
        out = np.empty(wx * wy * wz)
        _check(self.ctx, library().lbm_read_field_box(self.ctx, FIELDS[name], x0, y0, z0, wx, wy, wz, _ptr(out)))
        return out.reshape((wz, wy, wx))

    def fields(self) -> dict:
        rr, rb = self.field("rho_r"), self.field("rho_b")
        u = np.stack([self.field("ux"), self.field("uy"), self.field("uz")])
        return {"rho_r": rr, "rho_b": rb, "u": u, "rho": rr + rb, "phi": self.field("phi"), "p": self.field("p")}

    def field_box_noalloc(self, name: str, x0, y0, z0, wx, wy, wz) -> np.ndarray:
        """field_box through the entry point that allocates no device memory
        (lbm_read_field_box_noalloc)."""
        out = np.empty(wx * wy * wz)
        _check(self.ctx, library().lbm_read_field_box_noalloc(self.ctx, FIELDS[name], x0, y0, z0, wx, wy, wz,
                                                              _ptr(out)))
        return out.reshape((wz, wy, wx))

    def coarse_state_into(self, out, factor: int = 4, u_scale: float = 1.0):
        """Write the factor^3 block means of (phi, u / u_scale) into the device tensor `out`
        (FP32, shape (pd, ph, pw, 4) with the coarse lattice in its leading corner), on the
        lattice's stream (lbm_coarse_state)."""
        pd, ph, pw, c = out.shape
        if c != 4 or not out.is_contiguous() or out.dtype.itemsize != 4:
            raise ValueError("out must be a contiguous FP32 tensor of shape (pd, ph, pw, 4)")
        _check(self.ctx, library().lbm_coarse_state(self.ctx, int(factor), float(u_scale),
                                                    ctypes.c_void_p(out.data_ptr()), pd, ph, pw))

    def populations(self) -> np.ndarray:
        out = np.empty(2 * Q * self.n)
        _check(self.ctx, library().lbm_read_populations(self.ctx, _ptr(out)))
        return out.reshape((2, Q) + self.shape)

    def diagnostics(self, center=(0.0, 0.0, 0.0), r_in=0.0, r_out=1e30) -> dict:
        d = lbm_diag()
        st = library().lbm_diagnostics(self.ctx, float(center[0]), float(center[1]), float(center[2]), float(r_in),
                                       float(r_out), ctypes.byref(d))
        if st not in (LBM_OK, LBM_EUNSTABLE):
            _check(self.ctx, st)
        return {k: getattr(d, k) for k, _ in lbm_diag._fields_} | {"unstable": st == LBM_EUNSTABLE}

    def save_state(self) -> bytes:
        nb = library().lbm_state_bytes(self.ctx)
        buf = ctypes.create_string_buffer(nb)
        _check(self.ctx, library().lbm_save_state(self.ctx, buf, nb))
        return buf.raw

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self.ctx, library().lbm_load_state(self.ctx, buf, len(blob)))

    def last_step_kernel_ms(self) -> float:
        return float(library().lbm_last_step_kernel_ms(self.ctx))


class Batch:
    """Several lattices advanced together (lbm_batch_*): one step-kernel launch per step for
    all cases that share a storage type and tile shape.  ``cases[k]`` is a :class:`Lattice`
    view of case k (read-back, diagnostics); the batch owns the device memory."""

    def __init__(self, problems, storage: str = "f32", stream: Optional[int] = None, init: bool = True,
                 progress=None):
        n = len(problems)
        arr = (lbm_params * n)(*[params_from_problem(pb, storage) for pb in problems])
        self.handle = ctypes.c_void_p()
        st = library().lbm_batch_create(arr, n, ctypes.c_void_p(stream) if stream else None,
                                        ctypes.byref(self.handle))
        _check(None, st)
        self.cases = []
        for k, pb in enumerate(problems):
            ctx = ctypes.c_void_p(library().lbm_batch_case(self.handle, k))
            lat = Lattice(pb, storage=storage, init=False, _ctx=ctx)
            if init:
                if pb.rho_r is not None:
                    lat.init_fields(pb.rho_r, pb.rho_b, pb.u)
                else:  # fields made on demand, one case at a time
                    rr, rb, u = pb.field_fn(*pb.origin, pb.nx, pb.ny, pb.nz)
                    lat.init_fields(rr, rb, None if not np.any(u) else u)
                    del rr, rb, u
            self.cases.append(lat)
            if progress and (k + 1) % 8 == 0:
                progress(f"{k + 1}/{n} cases initialised")

    def _check(self, status):
        if status != LBM_OK:
            msg = library().lbm_batch_last_error(self.handle)
            raise LbmError(status, msg.decode() if msg else "")

    def autotune(self, trial_steps: int = 10):
        self._check(library().lbm_batch_autotune(self.handle, int(trial_steps)))

    def step(self, n: int = 1):
        self._check(library().lbm_batch_step(self.handle, int(n)))

    def sync(self):
        self._check(library().lbm_batch_sync(self.handle))

    def last_step_ms(self) -> float:
        return float(library().lbm_batch_last_step_ms(self.handle))

    def unstable_cases(self) -> list:
        """Indices of the cases the step kernel has flagged as unstable; they are no longer
        stepped (lbm_batch_unstable_cases)."""
        flags = (ctypes.c_int * len(self.cases))()
        n = library().lbm_batch_unstable_cases(self.handle, flags)
        if n < 0:
            self._check(LBM_EDEVICE)
        return [k for k in range(len(self.cases)) if flags[k]]

    @property
    def ncells(self) -> int:
        return sum(c.n for c in self.cases)

    def close(self):
        if getattr(self, "handle", None):
            for c in self.cases:
                c.ctx = None
            library().lbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sigma_from_A(A: float, nu: float) -> float:
    """Interfacial tension of the perturbation operator, Eq. (sigma), for the fluid of
    viscosity nu (lbm_sigma_from_A)."""
    return float(library().lbm_sigma_from_A(float(A), float(nu)))


def A_from_sigma(sigma: float, nu: float) -> float:
    """Surface-tension parameter giving the interfacial tension sigma, Eq. (sigma)
    inverted (lbm_A_from_sigma)."""
    return float(library().lbm_A_from_sigma(float(sigma), float(nu)))


def selftest_collide_host(problem, fr, fb, grad_phi, grad_rho):
    """The step's per-cell collision compiled for the host (diagnostic; no GPU)."""
    p = params_from_problem(problem)
    outr, outb = np.empty(Q), np.empty(Q)
    st = library().lbm_selftest_collide_host(ctypes.byref(p), _ptr(_arr(fr, Q)), _ptr(_arr(fb, Q)),
                                            _ptr(_arr(grad_phi, 3)), _ptr(_arr(grad_rho, 3)), _ptr(outr), _ptr(outb))
    _check(None, st)
    return outr, outb


def selftest_tile_sets_host(problem, tx: int, ty: int, storage: str = "f32") -> np.ndarray:
    """How the step's launches cover the tiles of tx x ty (diagnostic; no GPU): counts of shape
    (3, tiles_y, tiles_x) for the launch over all tiles, the interior tiles and the frame (whose
    split into launches depends on the storage type)."""
    p = params_from_problem(problem, storage)
    ntx, nty = -(-problem.nx // tx), -(-problem.ny // ty)
    counts = np.zeros(3 * ntx * nty, dtype=np.int32)
    st = library().lbm_selftest_tile_sets_host(ctypes.byref(p), int(tx), int(ty),
                                              counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    _check(None, st)
    return counts.reshape(3, nty, ntx)
