"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module states *problems*: lattice size, fluid properties, face types, body force,
inflow disk and the initial density/velocity fields.  It holds none of the method's
arithmetic (no equilibria, no moments, no collision); both implementations derive their
own lattice parameters from what is given here.

Initial profiles follow the paper's set-ups:
  * static droplet: tanh profile of width W = 4 around a sphere (Sec. III A);
  * Rayleigh-Taylor: flat interface at mid-height with a single-mode
    cos(2 pi x / W) + cos(2 pi y / W) displacement of amplitude 0.05 W (Sec. III C);
    the same tanh profile across it and a seeded 1e-4 relative density noise;
  * jet: domain full of the blue fluid at rest; red enters through an inflow disk on the
    z = 0 plane (Sec. IV A).
Per-cell noise is a counter-based draw on the global cell index, so that a window cut out
of a large domain sees the same numbers as the whole domain.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

PERIODIC, BOUNCEBACK, FREESLIP, OUTFLOW = 0, 1, 2, 3
FACE_NAMES = {PERIODIC: "periodic", BOUNCEBACK: "bounce-back", FREESLIP: "free-slip", OUTFLOW: "outflow"}


def splitmix64_uniform(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform draws on [-1, 1) from SplitMix64 (Steele, Lea & Flood 2014) used as a
    counter-based generator: value(n) = mix(seed + (n + 1) * golden_gamma)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counters.astype(np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 / 9007199254740992.0) - 1.0


@dataclasses.dataclass
class Problem:
    """A two-fluid problem on an nx x ny x nz lattice (x fastest)."""

    name: str
    nx: int
    ny: int
    nz: int
    rho_r0: float
    rho_b0: float
    nu_r: float
    nu_b: float
    A: Optional[float]  # surface-tension parameter; None: derived from sigma by each implementation
    beta: float
    faces: Sequence[int] = (PERIODIC,) * 6  # -x, +x, -y, +y, -z, +z
    force_model: int = 0  # 0: none, 1: F = (rho - rho_ref) g
    g: Sequence[float] = (0.0, 0.0, 0.0)
    rho_ref: float = 0.0
    inflow: bool = False
    xc: float = 0.0
    yc: float = 0.0
    diameter: float = 0.0
    u_in: float = 0.0
    noise_rel: float = 0.0
    seed: int = 0
    s: Optional[Sequence[float]] = None  # 27 relaxation rates or None for the defaults
    # interfacial tension, used when A is None: each implementation converts it with Eq. (sigma)
    # at the continuous (blue) phase's relaxation time (reading R6)
    sigma: Optional[float] = None
    # global frame (windows of a larger domain keep the global noise counter)
    gdims: Optional[Sequence[int]] = None
    origin: Sequence[int] = (0, 0, 0)
    # initial fields, shape (nz, ny, nx) and (3, nz, ny, nx)
    rho_r: Optional[np.ndarray] = None
    rho_b: Optional[np.ndarray] = None
    u: Optional[np.ndarray] = None
    steps: int = 0  # suggested number of steps for the workload
    field_fn: Optional[object] = dataclasses.field(default=None, repr=False)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def global_dims(self):
        return tuple(self.gdims) if self.gdims is not None else (self.nx, self.ny, self.nz)

    def window(self, x0: int, y0: int, z0: int, wx: int, wy: int, wz: int) -> "Problem":
        """Sub-box [x0, x0+wx) x [y0, y0+wy) x [z0, z0+wz) of this problem.

        Faces that are cut by the window become periodic (both cut) or bounce-back (one
        cut); cells further than 2 steps from a cut face per step taken are unaffected by
        the choice, because one step reads at most two cells away."""
        assert self.field_fn is not None, "window() needs a problem built by a generator"
        dims = (self.nx, self.ny, self.nz)
        lo = (x0, y0, z0)
        ext = (wx, wy, wz)
        faces = list(self.faces)
        for d in range(3):
            if lo[d] == 0 and ext[d] == dims[d]:
                continue
            if faces[2 * d] == PERIODIC:
                faces[2 * d] = faces[2 * d + 1] = PERIODIC
                continue
            if lo[d] != 0:
                faces[2 * d] = BOUNCEBACK
            if lo[d] + ext[d] != dims[d]:
                faces[2 * d + 1] = BOUNCEBACK
        gx0, gy0, gz0 = (self.origin[0] + x0, self.origin[1] + y0, self.origin[2] + z0)
        sub = dataclasses.replace(
            self,
            name=f"{self.name}[{x0}:{x0 + wx},{y0}:{y0 + wy},{z0}:{z0 + wz}]",
            nx=wx, ny=wy, nz=wz,
            faces=tuple(faces),
            xc=self.xc - x0, yc=self.yc - y0,
            inflow=self.inflow and z0 == 0,
            gdims=self.global_dims,
            origin=(gx0, gy0, gz0),
            rho_r=None, rho_b=None, u=None,
        )
        sub.rho_r, sub.rho_b, sub.u = self.field_fn(gx0, gy0, gz0, wx, wy, wz)
        return sub

    def with_fields(self) -> "Problem":
        if self.rho_r is None:
            self.rho_r, self.rho_b, self.u = self.field_fn(*self.origin, self.nx, self.ny, self.nz)
        return self


def _grid(x0, y0, z0, wx, wy, wz):
    z, y, x = np.meshgrid(np.arange(z0, z0 + wz, dtype=np.float64), np.arange(y0, y0 + wy, dtype=np.float64),
                          np.arange(x0, x0 + wx, dtype=np.float64), indexing="ij")
    return x, y, z


def static_droplet(n: int = 32, radius: float = 8.0, rho_r0: float = 1.0, rho_b0: float = 1.0,
                   nu: float = 1.0 / 6.0, A: float = 0.01, beta: float = 0.7, width: float = 4.0,
                   center: Optional[Sequence[float]] = None, dims: Optional[Sequence[int]] = None,
                   semi_axes: Optional[Sequence[float]] = None, steps: int = 200,
                   nu_b: Optional[float] = None) -> Problem:
    """Red droplet in blue, all faces periodic (Sec. III A).  With ``semi_axes`` the
    droplet is the prolate spheroid of the oscillation test (Sec. III B).  ``nu`` is the
    viscosity of both phases unless ``nu_b`` gives the blue one."""
    nx, ny, nz = dims if dims is not None else (n, n, n)
    c = center if center is not None else ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)

    def fields(x0, y0, z0, wx, wy, wz):
        x, y, z = _grid(x0, y0, z0, wx, wy, wz)
        if semi_axes is None:
            r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
            d = r - radius
        else:
            a, b, cc = semi_axes
            s = np.sqrt(((x - c[0]) / a) ** 2 + ((y - c[1]) / b) ** 2 + ((z - c[2]) / cc) ** 2)
            d = (s - 1.0) * min(a, b, cc)
        t = np.tanh(2.0 * d / width)
        return 0.5 * rho_r0 * (1.0 - t), 0.5 * rho_b0 * (1.0 + t), np.zeros((3, wz, wy, wx))

    return Problem(name="static_droplet", nx=nx, ny=ny, nz=nz, rho_r0=rho_r0, rho_b0=rho_b0, nu_r=nu,
                   nu_b=nu if nu_b is None else nu_b, A=A, beta=beta, steps=steps, field_fn=fields).with_fields()


def oscillating_droplet(nu: float, A: float, steps: int = 10000) -> Problem:
    """The oscillation test of Sec. III B: a 41^3 periodic lattice with a prolate spheroid of
    semi-axes 15, 11, 11 at the centre, density ratio 4 (the red droplet rho_r0 = 1 in
    rho_b0 = 0.25, reading R19), nu in both phases, the printed relaxation rates, beta = 0.7."""
    pb = static_droplet(n=41, rho_r0=1.0, rho_b0=0.25, nu=nu, A=A, beta=0.7, semi_axes=(15.0, 11.0, 11.0),
                        steps=steps)
    pb.s = None
    pb.name = f"oscillating_nu{nu:g}_A{A:g}"
    return pb


def laplace_droplet(radius: float, A: float, steps: int = 80000) -> Problem:
    """The Laplace-law test of Sec. III A (its table of R, A and E): an 85^3 periodic
    lattice, a red droplet of radius R at the centre in blue, interface width 4, density
    ratio 1.5, nu = 1e-3 in both phases, no gravity, 80 000 steps.  beta = 0.7 (the paper
    gives none)."""
    pb = static_droplet(n=85, radius=radius, rho_r0=1.5, rho_b0=1.0, nu=1e-3, A=A, beta=0.7, width=4.0, steps=steps)
    pb.name = f"laplace_R{radius:g}_A{A:g}"
    return pb


def stability_envelope(steps: int = 20000):
    """Static droplets at the ends of the stable ranges the paper states (Sec. V): density
    ratios gamma = rho_r / rho_b up to 1000 at nu_r = nu_b = 1e-3, and viscosity ratios
    eta = nu_r / nu_b up to 1000 at gamma = 1.5.  48^3, R = 12, width 4, beta = 0.7, with
    A = 1e-2 and 4e-4 (the surface tensions of Sec. III A).

    The paper does not say which phase is heavy or which viscosity changes.  The blue phase
    sets the pressure scale of the model (p = rho_b / 3 in both phases at rest), so the heavy
    droplet is red (rho_r0 = gamma, rho_b0 = 1): a light ambient of rho_b0 = 1/gamma would
    have a pressure below the Laplace jump at these A.  The viscosity ratio lowers the
    blue viscosity (nu_b = 1e-3 / eta): raising nu_r to 0.1 or 1 leaves the range where the
    printed relaxation rates are stable for a fluid at rest (about nu < 0.1)."""
    cases = []
    for gamma in (10.0, 100.0, 1000.0):
        for A in (1e-2, 4e-4):
            pb = static_droplet(n=48, radius=12.0, rho_r0=gamma, rho_b0=1.0, nu=1e-3, A=A, beta=0.7, width=4.0,
                                steps=steps)
            pb.name = f"envelope_gamma{gamma:g}_A{A:g}"
            cases.append(pb)
    for eta in (10.0, 100.0, 1000.0):
        pb = static_droplet(n=48, radius=12.0, rho_r0=1.5, rho_b0=1.0, nu=1e-3, nu_b=1e-3 / eta, A=1e-2, beta=0.7,
                            width=4.0, steps=steps)
        pb.name = f"envelope_eta{eta:g}"
        cases.append(pb)
    return cases


def rayleigh_taylor(width: int = 128, height: Optional[int] = None, atwood: float = 0.5, g: float = 1e-5,
                    reynolds: float = 256.0, beta: float = 0.7, noise: float = 1e-4, seed: int = 1,
                    iface_width: float = 4.0, steps: int = 20000) -> Problem:
    """Single-mode Rayleigh-Taylor set-up of Sec. III C on W x W x 4W.

    Heavy red (rho_r0) fills z below the perturbed mid-plane, light blue above; the body
    force F = (rho - (rho_r0 + rho_b0)/2) (0, 0, g) pushes the heavy fluid towards +z, so
    the heavy fluid lies on top with respect to the effective gravity.  Walls at both z
    ends are no-slip, the sides periodic.  Re = sqrt(W g) W / nu."""
    W = width
    H = height if height is not None else 4 * W
    rho_b0 = 1.0
    rho_r0 = rho_b0 * (1.0 + atwood) / (1.0 - atwood)
    nu = math.sqrt(W * g) * W / reynolds
    zmid = (H - 1) / 2.0
    ncell_global = (W, W, H)

    def fields(x0, y0, z0, wx, wy, wz):
        x, y, z = _grid(x0, y0, z0, wx, wy, wz)
        zi = zmid + 0.05 * W * (np.cos(2 * np.pi * x / W) + np.cos(2 * np.pi * y / W))
        t = np.tanh(2.0 * (z - zi) / iface_width)
        rr = 0.5 * rho_r0 * (1.0 - t)
        rb = 0.5 * rho_b0 * (1.0 + t)
        if noise:
            gidx = ((z.astype(np.int64) * ncell_global[1] + y.astype(np.int64)) * ncell_global[0] + x.astype(np.int64))
            rr = rr * (1.0 + noise * splitmix64_uniform(seed, 2 * gidx))
            rb = rb * (1.0 + noise * splitmix64_uniform(seed, 2 * gidx + 1))
        return rr, rb, np.zeros((3, wz, wy, wx))

    return Problem(name="rayleigh_taylor", nx=W, ny=W, nz=H, rho_r0=rho_r0, rho_b0=rho_b0, nu_r=nu, nu_b=nu,
                   A=0.0, beta=beta, faces=(PERIODIC, PERIODIC, PERIODIC, PERIODIC, BOUNCEBACK, BOUNCEBACK),
                   force_model=1, g=(0.0, 0.0, g), rho_ref=0.5 * (rho_r0 + rho_b0), seed=seed, steps=steps,
                   field_fn=fields).with_fields()


def jet(nx: int = 256, ny: int = 256, nz: int = 1024, diameter: float = 16.0, u_in: float = 0.04,
        gamma: float = 1.6, nu_c: float = 1.8e-4, eta: float = 1.0, weber: float = 220.0, froude: float = 8.5,
        A: Optional[float] = None, beta: float = 0.7, noise_rel: float = 0.01, seed: int = 3,
        steps: int = 30000, fields: bool = True, lateral: int = PERIODIC) -> Problem:
    """Liquid jet into an immiscible liquid (Sec. IV A): inflow disk on z = 0 with
    free-slip elsewhere on that plane, convective outflow on the last plane, and sides that
    are periodic or, with ``lateral=FREESLIP``, the free-slip walls of the paper's set-up.
    rho_j = 1; sigma from We = rho_j u^2 D / sigma; g from Fr = u^2 / (g D); nu_j = eta nu_c.
    Unless ``A`` is given, the problem carries sigma and each implementation derives the
    surface-tension parameter from it at the continuous phase's relaxation time (Eq. (sigma),
    reading R6)."""
    rho_r0 = 1.0
    rho_b0 = rho_r0 / gamma
    nu_j = eta * nu_c
    sigma = rho_r0 * u_in ** 2 * diameter / weber
    g = u_in ** 2 / (froude * diameter)

    def make_fields(x0, y0, z0, wx, wy, wz):
        shape = (wz, wy, wx)
        return np.zeros(shape), np.full(shape, rho_b0), np.zeros((3,) + shape)

    pb = Problem(name="jet", nx=nx, ny=ny, nz=nz, rho_r0=rho_r0, rho_b0=rho_b0, nu_r=nu_j, nu_b=nu_c, A=A,
                 sigma=None if A is not None else sigma,
                 beta=beta, faces=(lateral,) * 4 + (FREESLIP, OUTFLOW), force_model=1,
                 g=(0.0, 0.0, g), rho_ref=rho_b0, inflow=True, xc=(nx - 1) / 2.0, yc=(ny - 1) / 2.0,
                 diameter=diameter, u_in=u_in, noise_rel=noise_rel, seed=seed, steps=steps,
                 field_fn=make_fields)
    return pb.with_fields() if fields else pb


# --- dimensionless groups of the jet (Sec. IV B, Eqs. (densityRatio)-(Froude)) -------------

def jet_groups(D: float, u: float, rho_j: float, rho_c: float, sigma: float, nu_j: float, nu_c: float,
               g: float) -> dict:
    """gamma, eta, Re, We, Fr and Oh = We^(1/2)/Re of a jet given in lattice units."""
    Re = u * D / nu_j
    We = rho_j * u * u * D / sigma
    return {"gamma": rho_j / rho_c, "eta": nu_j / nu_c, "Re": Re, "We": We, "Fr": u * u / (g * D),
            "Oh": math.sqrt(We) / Re}


def breakup_regime(Re: float, Oh: float) -> str:
    """Regime label from the transition criteria Oh = 2.8/Re (I/II) and Oh = 22/Re
    (II/III) of Sec. IV C (dripping is not separated from Regime I)."""
    if Oh * Re < 2.8:
        return "I"
    if Oh * Re < 22.0:
        return "II"
    return "III"


def regime_sweep(ncases: int = 64, seed: int = 4, sizes=(96, 112, 128, 144, 160), diameters=(8, 16),
                 fields: bool = False) -> list:
    """Regime-map sweep of uneven jet cases (Sec. IV C): per case, drawn from a seeded
    generator, nozzle D uniform on the integers of `diameters`, width L from `sizes` with
    height 4 L, Re log-uniform on [100, 3400], Oh log-uniform on [0.005, 0.5], gamma
    uniform on [1.2, 2.0]; u = 0.04, nu_j = nu_c = u D / Re, We = (Oh Re)^2, Fr = 8.5, 1 %
    inflow noise.  Fields are made on demand unless `fields`."""
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(ncases):
        D = int(rng.integers(diameters[0], diameters[1] + 1))
        L = int(sizes[int(rng.integers(0, len(sizes)))])
        Re = float(np.exp(rng.uniform(np.log(100.0), np.log(3400.0))))
        Oh = float(np.exp(rng.uniform(np.log(0.005), np.log(0.5))))
        gamma = float(rng.uniform(1.2, 2.0))
        u = 0.04
        pb = jet(nx=L, ny=L, nz=4 * L, diameter=float(D), u_in=u, gamma=gamma, nu_c=u * D / Re, eta=1.0,
                 weber=(Oh * Re) ** 2, froude=8.5, noise_rel=0.01, seed=seed * 1000 + k, steps=5000, fields=fields)
        pb.name = f"sweep{k:02d}_L{L}_D{D}_Re{Re:.0f}_Oh{Oh:.3f}_g{gamma:.2f}"
        pb.regime = breakup_regime(Re, Oh)
        cases.append(pb)
    return cases


def paper_rayleigh_taylor(reynolds: float) -> Problem:
    """The Rayleigh-Taylor runs of Sec. III C at the paper's size: 128 x 128 x 512,
    At = 0.5, (W g)^(1/2) = 0.04, no interfacial tension, equal viscosities from Re, the
    single-mode perturbation and no noise.  t* = t / (W/g)^(1/2), 3200 steps per unit."""
    W = 128
    g = 0.04 ** 2 / W
    pb = rayleigh_taylor(width=W, atwood=0.5, g=g, reynolds=float(reynolds), noise=0.0)
    pb.name = f"paper_rayleigh_taylor_Re{reynolds:g}"
    pb.t_unit = math.sqrt(W / g)
    return pb


# Lattice-unit parameters of the paper's liquid-liquid jets (Sec. IV B, Table III; Sec. IV C,
# Table IV): inlet diameter D, inlet speed u, rho_c (rho_j = 1), sigma, nu_j, nu_c, g, and
# the 8D x 8D x 20D lattice.
PAPER_JETS = {
    "ref": dict(D=25, u=0.10, rho_c=0.70, sigma=1.1e-3, nu_j=7.4e-4, nu_c=1.8e-4, g=4.7e-5),
    "case1": dict(D=15, u=0.05, rho_c=0.70, sigma=9.1e-3, nu_j=1.6e-3, nu_c=3.9e-4, g=2.0e-5),
    "case2": dict(D=30, u=0.10, rho_c=0.70, sigma=3.0e-5, nu_j=8.8e-4, nu_c=2.1e-4, g=3.9e-5),
}


def paper_jet(case: str = "ref", fields: bool = True, lateral: int = FREESLIP) -> Problem:
    """One of the paper's jets at its own size (Sec. IV B-C): "ref" (200 x 200 x 500, sinuous
    breakup, Regime II), "case1" (120 x 120 x 300, varicose, Regime I) or "case2"
    (240 x 240 x 600, atomisation, Regime III), with the paper's free-slip lateral walls
    (Sec. IV A).  No inflow noise: the paper adds no perturbation, the instability grows from
    the flow itself.  sigma is converted to A at the continuous phase's relaxation time."""
    c = PAPER_JETS[case]
    D, u = c["D"], c["u"]
    pb = jet(nx=8 * D, ny=8 * D, nz=20 * D, diameter=float(D), u_in=u, gamma=1.0 / c["rho_c"], nu_c=c["nu_c"],
             eta=c["nu_j"] / c["nu_c"], weber=u * u * D / c["sigma"], froude=u * u / (c["g"] * D), noise_rel=0.0,
             fields=fields, lateral=lateral)
    pb.name = f"paper_jet_{case}_{8 * D}x{8 * D}x{20 * D}"
    pb.t_unit = D / u  # steps per unit of t* = t u / D
    return pb


UNIT_RATES = (0.0,) * 4 + (1.0,) * 23


def cfg_static_droplet(steps: int = 200) -> Problem:
    """32^3 static droplet, R = 8 centred, density ratio 1, tau = 1 in both phases,
    A = 0.01, beta = 0.7.  tau = 1 is read as every non-conserved relaxation rate equal to
    1/tau: Suga's rates make the method linearly unstable at rest for nu >~ 0.1."""
    pb = static_droplet(n=32, radius=8.0, nu=1.0 / 6.0, A=0.01, beta=0.7, steps=steps)
    pb.s = UNIT_RATES
    pb.name = "static_droplet_32"
    return pb


def cfg_rayleigh_taylor(steps: int = 20000) -> Problem:
    """128 x 128 x 512 Rayleigh-Taylor, At = 0.5, g = 1e-5, Re = 256, seeded 1e-4 noise."""
    pb = rayleigh_taylor(width=128, atwood=0.5, g=1e-5, reynolds=256.0, noise=1e-4, seed=1, steps=steps)
    pb.name = "rayleigh_taylor_128x128x512"
    return pb


def cfg_jet(steps: int = 30000) -> Problem:
    """256 x 256 x 1024 jet, D = 16, u = 0.04, nu = 1.8e-4 in both phases, gamma = 1.6,
    We = 220, Fr = 8.5, 1 % inflow noise."""
    pb = jet(nx=256, ny=256, nz=1024, diameter=16.0, u_in=0.04, gamma=1.6, nu_c=1.8e-4, eta=1.0, weber=220.0,
             froude=8.5, noise_rel=0.01, seed=3, steps=steps)
    pb.name = "jet_256x256x1024"
    return pb


def cfg_jet_walls(steps: int = 30000) -> Problem:
    """The jet of ``cfg_jet`` between free-slip lateral walls, as in the paper's own jet runs
    (Sec. IV A)."""
    pb = jet(nx=256, ny=256, nz=1024, diameter=16.0, u_in=0.04, gamma=1.6, nu_c=1.8e-4, eta=1.0, weber=220.0,
             froude=8.5, noise_rel=0.01, seed=3, steps=steps, lateral=FREESLIP)
    pb.name = "jet_walls_256x256x1024"
    return pb


def small_configs():
    """Parity-sized problems: the 32^3 static droplet, a droplet with Suga's rates at a
    viscosity where they are stable, a reduced Rayleigh-Taylor box and a reduced jet with
    the physics of the full-size workloads; and, for the local viscosity and the
    density-ratio terms, the reduced jet at the paper's viscosity ratio eta = 4.2 (Table III),
    a droplet with eta = 10 (nu_b = 1e-3), one with density ratio gamma = 10, and the reduced
    jet at eta = 4.2 between the free-slip lateral walls of the paper's jet set-up."""
    suga_drop = static_droplet(n=24, radius=6.0, rho_r0=1.5, rho_b0=1.0, nu=1.667e-2, A=0.01, beta=0.7)
    suga_drop.name = "droplet24_suga"
    eta_drop = static_droplet(n=24, radius=6.0, rho_r0=1.5, rho_b0=1.0, nu=1e-2, nu_b=1e-3, A=0.01, beta=0.7)
    eta_drop.name = "droplet24_eta10"
    gamma_drop = static_droplet(n=24, radius=6.0, rho_r0=10.0, rho_b0=1.0, nu=1e-2, A=0.01, beta=0.7)
    gamma_drop.name = "droplet24_gamma10"
    jet_eta = jet(nx=24, ny=24, nz=48, diameter=8.0, eta=4.2)
    jet_eta.name = "jet_small_eta4.2"
    jet_walls = jet(nx=24, ny=24, nz=48, diameter=8.0, eta=4.2, lateral=FREESLIP)
    jet_walls.name = "jet_small_walls"
    return {
        "droplet32": cfg_static_droplet(),
        "droplet24_suga": suga_drop,
        "rt_small": rayleigh_taylor(width=16, height=48, g=1e-4, reynolds=64.0),
        "jet_small": jet(nx=24, ny=24, nz=48, diameter=8.0),
        "droplet24_eta10": eta_drop,
        "droplet24_gamma10": gamma_drop,
        "jet_small_eta": jet_eta,
        "jet_small_walls": jet_walls,
    }
