"""Host-side measures on read-back fields (numpy, no GPU).

interface_position_error(phi_a, phi_b): how far apart two runs put the interface.  Over the
cells where run b sees the interface (|phi_b| < 0.9), the local displacement of the phase
field is |phi_a - phi_b| / |grad phi_b| in lattice units (phi changes by |grad phi| per lattice
unit across the interface, so a shift of the interface by d moves phi by d |grad phi|).
Returns the mean and the maximum over those cells.

Also: interface tracking of the paper's test problems (droplet half-axes, Rayleigh-Taylor
front positions, jet leading edge) and the parity measures used by the tests.
"""
from __future__ import annotations

import numpy as np


def interface_position_error(phi_a: np.ndarray, phi_b: np.ndarray, band: float = 0.9, periodic=(True, True, False),
                             min_grad: float = 1e-3) -> dict:
    """Interface displacement of field a relative to field b (arrays indexed [z, y, x]).

    periodic: per axis (x, y, z) whether central differences wrap.  Cells whose phase
    gradient is below min_grad (flat plateaus inside the band) are skipped."""
    if phi_a.shape != phi_b.shape:
        raise ValueError("fields differ in shape")
    grads = []
    for axis_xyz, per in zip((2, 1, 0), periodic):
        if per:
            d = 0.5 * (np.roll(phi_b, -1, axis=axis_xyz) - np.roll(phi_b, 1, axis=axis_xyz))
        else:
            d = np.gradient(phi_b, axis=axis_xyz)
        grads.append(d)
    gmag = np.sqrt(sum(g * g for g in grads))
    sel = (np.abs(phi_b) < band) & (gmag > min_grad)
    if not np.any(sel):
        return {"cells": 0, "mean_lu": 0.0, "max_lu": 0.0}
    disp = np.abs(phi_a[sel] - phi_b[sel]) / gmag[sel]
    return {"cells": int(sel.sum()), "mean_lu": float(disp.mean()), "max_lu": float(disp.max())}


def crossing(profile: np.ndarray, start: int, step: int = 1) -> float:
    """Position where a 1-D phase profile changes sign, searching from index `start` in
    direction `step` (+1 or -1); linear interpolation between the two cells around the
    change.  NaN if it never changes sign."""
    s0 = np.sign(profile[start])
    k = start
    n = profile.shape[0]
    while 0 <= k + step < n and np.sign(profile[k + step]) == s0:
        k += step
    if not 0 <= k + step < n:
        return float("nan")
    a, b = profile[k], profile[k + step]
    return float(k + step * a / (a - b))


def droplet_half_axes(phi: np.ndarray, center) -> tuple:
    """Half-lengths of a droplet (phi > 0 inside) along x, y and z through its centre
    (cell indices, arrays indexed [z, y, x]): the interface tracking of the oscillation
    test (Sec. III B)."""
    cx, cy, cz = (int(round(c)) for c in center)
    return (crossing(phi[cz, cy, :], cx) - cx, crossing(phi[cz, :, cx], cy) - cy, crossing(phi[:, cy, cx], cz) - cz)


def rt_front_positions(phi: np.ndarray) -> dict:
    """Rayleigh-Taylor front positions (Sec. III C) on a W x W x H lattice with the heavy
    fluid (phi > 0) at low z and the body force pushing it towards +z: the spike tip at the
    column (0, 0), the bubble tip at (W/2, W/2) and the saddle at (0, W/2) of the
    single-mode perturbation; each is the z where phi changes sign, searched from z = 0."""
    W = phi.shape[2]
    h = W // 2
    return {"spike": crossing(phi[:, 0, 0], 0), "bubble": crossing(phi[:, h, h], 0), "saddle": crossing(phi[:, h, 0], 0)}


def jet_leading_edge(phi: np.ndarray, threshold: float = 0.0) -> float:
    """Largest z (cell index) holding injected fluid (phi > threshold) anywhere in its plane:
    the leading edge of the jet (Sec. IV)."""
    planes = np.nonzero((phi > threshold).any(axis=(1, 2)))[0]
    return float(planes.max()) if planes.size else float("nan")


def relative_errors(got: dict, ref: dict) -> dict:
    """Parity measures of two field sets: e_rho = max|rho_a - rho_b| / max|rho_b| (also per
    colour, on the same scale), e_u = max|u_a - u_b| / max|u_b|."""
    rho_ref = ref["rho_r"] + ref["rho_b"]
    scale = float(np.abs(rho_ref).max())
    e = {k: float(np.abs(got[k] - ref[k]).max() / scale) for k in ("rho_r", "rho_b")}
    e["rho"] = float(np.abs(got["rho_r"] + got["rho_b"] - rho_ref).max() / scale)
    umag = float(np.abs(ref["u"]).max())
    du = float(np.abs(got["u"] - ref["u"]).max())
    e["u"] = du / umag if umag > 0 else du
    e["umax_ref"] = umag
    return e


def laplace_error(diag: dict, A: float, nu: float, rho_r0: float) -> dict:
    """Laplace-law measurement of Sec. III A from the lattice's FP64 diagnostics (mean
    pressure p_in within R/2 of the centre and p_out beyond R + 6): Delta p = p_in - p_out,
    the radius from the red mass, R = (3 m_r / (4 pi rho_r0))^(1/3), the measured tension
    sigma_lap = Delta p R / 2 (Eq. (lap)), the predicted sigma_th = (4/9) A (3 nu + 1/2)
    (Eq. (sigma)) and the error E = |sigma_th - sigma_lap| / sigma_th."""
    dp = diag["p_in"] - diag["p_out"]
    radius = (3.0 * diag["mass_r"] / (4.0 * np.pi * rho_r0)) ** (1.0 / 3.0)
    sigma_lap = dp * radius / 2.0
    sigma_th = 4.0 / 9.0 * A * (3.0 * nu + 0.5)
    return {"dp": dp, "radius": radius, "sigma_lap": sigma_lap, "sigma_th": sigma_th,
            "E": abs(sigma_th - sigma_lap) / sigma_th}


def extrema_times(ts, values) -> list:
    """Times of the interior local extrema of a sampled signal, each refined by the vertex of
    the parabola through it and its two neighbours (uniform sampling)."""
    ts = np.asarray(ts, dtype=float)
    v = np.asarray(values, dtype=float)
    out = []
    for k in range(1, len(v) - 1):
        if (v[k] - v[k - 1]) * (v[k + 1] - v[k]) < 0:
            den = v[k - 1] - 2.0 * v[k] + v[k + 1]
            off = 0.5 * (v[k - 1] - v[k + 1]) / den if den != 0 else 0.0
            out.append(float(ts[k] + off * (ts[1] - ts[0])))
    return out


def oscillation_period(ts, values, skip: int = 1) -> float:
    """Period of a decaying oscillation: twice the mean time between successive extrema,
    leaving out the first ``skip`` half-periods (the largest, least linear amplitude); NaN
    when fewer than skip + 1 half-periods were seen."""
    e = extrema_times(ts, values)
    halves = np.diff(e)[skip:]
    return float(2.0 * halves.mean()) if len(halves) else float("nan")


def equivalent_radius(phi: np.ndarray) -> float:
    """Radius of the sphere with the volume of the cells where phi > 0 (the droplet)."""
    return float((3.0 * float((np.asarray(phi) > 0).sum()) / (4.0 * np.pi)) ** (1.0 / 3.0))


def jet_blobs(phi: np.ndarray, inlet_plane: int = 0) -> dict:
    """Connected regions of the jet fluid (phi > 0, 26-connected, x and y periodic) of a
    jet lattice [z][y][x]: the column (the region that touches the inlet plane) and the
    detached drops.  Returns the column's length (its largest z + 1), the drops' equivalent
    diameters (6 V / pi)^(1/3) sorted in decreasing order, and the column's cross-section
    radius sqrt(area / pi) per plane."""
    from scipy import ndimage

    mask = phi > 0.0
    lab, n = ndimage.label(mask, structure=np.ones((3, 3, 3), dtype=bool))
    if n == 0:
        return {"column_length": 0.0, "drops": np.zeros(0), "radius": np.zeros(phi.shape[0])}
    # regions that touch across the periodic x and y faces are one region
    parent = np.arange(n + 1)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a_face, b_face in ((lab[:, :, 0], lab[:, :, -1]), (lab[:, 0, :], lab[:, -1, :])):
        both = (a_face > 0) & (b_face > 0)
        for a, b in zip(a_face[both], b_face[both]):
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(k) for k in range(n + 1)])
    lab = roots[lab]
    sizes = np.bincount(lab.ravel(), minlength=n + 1)
    col = set(np.unique(lab[inlet_plane][lab[inlet_plane] > 0]).tolist())
    drops = [sizes[k] for k in np.unique(lab[lab > 0]) if k not in col]
    colmask = np.isin(lab, list(col)) if col else np.zeros_like(mask)
    zs = np.nonzero(colmask.any(axis=(1, 2)))[0]
    return {"column_length": float(zs.max() + 1) if zs.size else 0.0,
            "drops": np.sort((6.0 * np.asarray(drops, dtype=float) / np.pi) ** (1.0 / 3.0))[::-1],
            "radius": np.sqrt(colmask.sum(axis=(1, 2)) / np.pi)}


def jet_head_and_stem(radius: np.ndarray, column_length: float, D: float) -> tuple:
    """Mushroom-head measure of a jet column (Sec. IV B): the largest cross-section radius
    in the leading 40 % of the column and the radius 2 D from the inlet, both over the inlet
    radius D/2 (nan when the column is shorter than 2 D)."""
    L = int(column_length)
    if L <= 2 * D:
        return float("nan"), float("nan")
    return float(radius[int(0.6 * L):L].max() / (D / 2)), float(radius[int(2 * D)] / (D / 2))


def jet_axis_offset(phi: np.ndarray, column_length: float, D: float) -> float:
    """Largest distance, over the planes of the column, between the centroid of the jet fluid
    (phi > 0) in the plane and the inlet axis, in units of D: 0 for an axisymmetric column,
    of order D once it winds (Sec. IV B-C)."""
    nz, ny, nx = phi.shape
    yy, xx = np.mgrid[0:ny, 0:nx]
    xc, yc = (nx - 1) / 2.0, (ny - 1) / 2.0
    off = 0.0
    for z in range(0, int(column_length)):
        m = phi[z] > 0.0
        if m.sum() >= 4:
            off = max(off, float(np.hypot(xx[m].mean() - xc, yy[m].mean() - yc)))
    return off / D


def interface_area(phi: np.ndarray) -> int:
    """Number of cell faces across which phi changes sign: a measure of the interface area
    (in lattice units squared, staircase-counted) that grows as the interface folds."""
    m = phi > 0.0
    return int((m[1:] != m[:-1]).sum() + (m[:, 1:] != m[:, :-1]).sum() + (m[:, :, 1:] != m[:, :, :-1]).sum())
