"""FP64 CPU oracle of the D3Q27 colour-fluid LBM step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The library it wraps, ``liblbm_oracle.so``, is compiled from
``lbm_oracle.c`` with gcc; it shares nothing with the HIP implementation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")
Q = 27


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc (OpenMP over cells, FP64, no fast-math)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("rho_r0", ctypes.c_double), ("rho_b0", ctypes.c_double),
        ("nu_r", ctypes.c_double), ("nu_b", ctypes.c_double),
        ("A", ctypes.c_double), ("beta", ctypes.c_double),
        ("s", ctypes.c_double * Q),
        ("face", ctypes.c_int * 6),
        ("force_model", ctypes.c_int),
        ("g", ctypes.c_double * 3),
        ("rho_ref", ctypes.c_double),
        ("inflow", ctypes.c_int),
        ("xc", ctypes.c_double), ("yc", ctypes.c_double), ("diameter", ctypes.c_double),
        ("u_in", ctypes.c_double), ("noise_rel", ctypes.c_double),
        ("seed", ctypes.c_ulonglong),
        ("gnx", ctypes.c_int), ("gny", ctypes.c_int), ("gnz", ctypes.c_int),
        ("ox", ctypes.c_int), ("oy", ctypes.c_int), ("oz", ctypes.c_int),
        ("gphi_cut", ctypes.c_double),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        L.oracle_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_void_p)]
        L.oracle_create.restype = ctypes.c_int
        L.oracle_destroy.argtypes = [ctypes.c_void_p]
        L.oracle_init.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.oracle_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.oracle_fields.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.oracle_populations.argtypes = [ctypes.c_void_p, _D]
        L.oracle_set_populations.argtypes = [ctypes.c_void_p, _D]
        L.oracle_step_count.argtypes = [ctypes.c_void_p]
        L.oracle_step_count.restype = ctypes.c_longlong
        L.oracle_get_matrices.argtypes = [ctypes.c_void_p, _D, _D]
        L.oracle_get_lattice.argtypes = [ctypes.POINTER(ctypes.c_int), _D, _D]
        L.oracle_get_varphi.argtypes = [ctypes.c_double, _D]
        L.oracle_alpha_r.argtypes = [ctypes.c_void_p]
        L.oracle_alpha_r.restype = ctypes.c_double
        L.oracle_relaxation_diag.argtypes = [ctypes.c_void_p, ctypes.c_double, _D]
        L.oracle_equilibrium.argtypes = [ctypes.c_double] * 4 + [_D, ctypes.c_double, _D, _D]
        L.oracle_colour_equilibrium.argtypes = [ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_forcing_velocity_space.argtypes = [_D, _D, _D]
        L.oracle_perturbation.argtypes = [ctypes.c_double, ctypes.c_double, _D, _D]
        L.oracle_recolour.argtypes = [ctypes.c_double] * 5 + [_D, _D, _D, _D]
        L.oracle_collide_cell.argtypes = [ctypes.c_void_p, _D, _D, _D, _D, _D, _D, _D]
        L.oracle_gradient.argtypes = [ctypes.c_void_p, _D, _D]
        L.oracle_A_from_sigma.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_A_from_sigma.restype = ctypes.c_double
        L.oracle_noise.argtypes = [ctypes.c_ulonglong, ctypes.c_ulonglong]
        L.oracle_noise.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _vec(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


# Reading R7: the interface normal is undefined where |grad phi| <= this, the FP64 noise
# floor (rounding leaves ~1e-17 at symmetry points, where the exact gradient is 0).
GPHI_CUT = 1e-12


def params_from_problem(pb, gphi_cut: float = GPHI_CUT) -> _Params:
    """Oracle parameters of a problem.  ``gphi_cut`` is the |grad phi| at and below which
    the interface normal is taken as undefined (reading R7)."""
    p = _Params()
    p.nx, p.ny, p.nz = pb.nx, pb.ny, pb.nz
    p.rho_r0, p.rho_b0, p.nu_r, p.nu_b = pb.rho_r0, pb.rho_b0, pb.nu_r, pb.nu_b
    p.A = pb.A if pb.A is not None else lib().oracle_A_from_sigma(float(pb.sigma), float(pb.nu_b))
    p.beta = pb.beta
    if pb.s is not None:
        for j in range(Q):
            p.s[j] = pb.s[j]
    for k in range(6):
        p.face[k] = int(pb.faces[k])
    p.force_model = int(pb.force_model)
    for a in range(3):
        p.g[a] = pb.g[a]
    p.rho_ref = pb.rho_ref
    p.inflow = 1 if pb.inflow else 0
    p.xc, p.yc, p.diameter, p.u_in, p.noise_rel = pb.xc, pb.yc, pb.diameter, pb.u_in, pb.noise_rel
    p.seed = int(pb.seed)
    p.gnx, p.gny, p.gnz = pb.global_dims
    p.ox, p.oy, p.oz = pb.origin
    p.gphi_cut = float(gphi_cut)
    return p


class Oracle:
    """A running FP64 simulation of a :class:`workloads.Problem`."""

    def __init__(self, problem, init: bool = True, gphi_cut: float = GPHI_CUT):
        self.pb = problem
        self._p = params_from_problem(problem, gphi_cut)
        h = ctypes.c_void_p()
        rc = lib().oracle_create(ctypes.byref(self._p), ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"oracle_create failed with code {rc}")
        self._h = h
        self.n = problem.ncells
        if init:
            self.init(problem.rho_r, problem.rho_b, problem.u)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_destroy(h)
            self._h = None

    def init(self, rho_r, rho_b, u=None):
        rr = _vec(rho_r, self.n)
        rb = _vec(rho_b, self.n)
        uu = _vec(u, 3 * self.n) if u is not None else None
        lib().oracle_init(self._h, _ptr(rr), _ptr(rb), _ptr(uu) if uu is not None else None)

    def step(self, n: int = 1):
        lib().oracle_step(self._h, int(n))

    @property
    def steps_done(self) -> int:
        return int(lib().oracle_step_count(self._h))

    @property
    def alpha_r(self) -> float:
        return float(lib().oracle_alpha_r(self._h))

    def fields(self) -> dict:
        """rho_r, rho_b, u (3, nz, ny, nx), phi and rho at the current time."""
        shape = (self.pb.nz, self.pb.ny, self.pb.nx)
        rr = np.empty(self.n)
        rb = np.empty(self.n)
        u = np.empty(3 * self.n)
        lib().oracle_fields(self._h, _ptr(rr), _ptr(rb), _ptr(u))
        rr, rb, u = rr.reshape(shape), rb.reshape(shape), u.reshape((3,) + shape)
        return {"rho_r": rr, "rho_b": rb, "u": u, "rho": rr + rb, "phi": (rr - rb) / (rr + rb)}

    def populations(self) -> np.ndarray:
        out = np.empty(2 * Q * self.n)
        lib().oracle_populations(self._h, _ptr(out))
        return out.reshape(2, Q, self.pb.nz, self.pb.ny, self.pb.nx)

    def set_populations(self, f: np.ndarray):
        a = _vec(f, 2 * Q * self.n)
        lib().oracle_set_populations(self._h, _ptr(a))

    def gradient(self, field) -> np.ndarray:
        fld = _vec(field, self.n)
        out = np.empty(3 * self.n)
        lib().oracle_gradient(self._h, _ptr(fld), _ptr(out))
        return out.reshape(3, self.pb.nz, self.pb.ny, self.pb.nx)

    def matrices(self):
        M = np.empty(Q * Q)
        Mi = np.empty(Q * Q)
        lib().oracle_get_matrices(self._h, _ptr(M), _ptr(Mi))
        return M.reshape(Q, Q), Mi.reshape(Q, Q)

    def relaxation(self, snu: float) -> np.ndarray:
        K = np.empty(Q)
        lib().oracle_relaxation_diag(self._h, float(snu), _ptr(K))
        return K

    def collide_cell(self, fr, fb, grad_phi, grad_rho, F):
        fr, fb = _vec(fr, Q), _vec(fb, Q)
        gp, gr, FF = _vec(grad_phi, 3), _vec(grad_rho, 3), _vec(F, 3)
        outr, outb = np.empty(Q), np.empty(Q)
        lib().oracle_collide_cell(self._h, _ptr(fr), _ptr(fb), _ptr(gp), _ptr(gr), _ptr(FF), _ptr(outr), _ptr(outb))
        return outr, outb


# ---- per-cell operators, for unit tests ----------------------------------------------

def lattice():
    c = (ctypes.c_int * (3 * Q))()
    w = np.empty(Q)
    B = np.empty(Q)
    lib().oracle_get_lattice(c, _ptr(w), _ptr(B))
    return np.array(list(c), dtype=np.int64).reshape(Q, 3), w, B


def varphi(alpha: float) -> np.ndarray:
    out = np.empty(Q)
    lib().oracle_get_varphi(float(alpha), _ptr(out))
    return out


def equilibrium(rho_r, rho_b, alpha_r, alpha_b, u, nubar, grad_rho) -> np.ndarray:
    out = np.empty(Q)
    uu, gr = _vec(u, 3), _vec(grad_rho, 3)
    lib().oracle_equilibrium(float(rho_r), float(rho_b), float(alpha_r), float(alpha_b), _ptr(uu), float(nubar),
                             _ptr(gr), _ptr(out))
    return out


def colour_equilibrium(rho_k, alpha_k, u) -> np.ndarray:
    out = np.empty(Q)
    uu = _vec(u, 3)
    lib().oracle_colour_equilibrium(float(rho_k), float(alpha_k), _ptr(uu), _ptr(out))
    return out


def forcing_velocity_space(u, F) -> np.ndarray:
    out = np.empty(Q)
    uu, FF = _vec(u, 3), _vec(F, 3)
    lib().oracle_forcing_velocity_space(_ptr(uu), _ptr(FF), _ptr(out))
    return out


def perturbation(A, grad_phi, f, gphi_cut: float = GPHI_CUT) -> np.ndarray:
    out = _vec(f, Q).copy()
    gp = _vec(grad_phi, 3)
    lib().oracle_perturbation(float(A), float(gphi_cut), _ptr(gp), _ptr(out))
    return out


def recolour(rho_r, rho_b, beta, alpha_bar, grad_phi, f, gphi_cut: float = GPHI_CUT):
    fr, fb = np.empty(Q), np.empty(Q)
    gp, ff = _vec(grad_phi, 3), _vec(f, Q)
    lib().oracle_recolour(float(rho_r), float(rho_b), float(beta), float(alpha_bar), float(gphi_cut), _ptr(gp),
                          _ptr(ff), _ptr(fr), _ptr(fb))
    return fr, fb


def noise(seed: int, counter: int) -> float:
    return float(lib().oracle_noise(int(seed), int(counter)))
