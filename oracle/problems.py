"""Initial conditions of the benchmark problems (oracle, test infrastructure).

Each problem fixes the domain, the adiabatic index, whether artificial
viscosity is used, and the initial velocity, density and pressure (Sec. 6.1).
Velocities are interpolated at the Q2 nodes, the specific internal energy
e = p / ((gamma - 1) rho) (eq. EOS) at the Q1 nodes, positions are the node
coordinates, and rho0 = 1 everywhere except in the triple-point problem.

Readings where the paper is silent or garbled:

* Gresho: the middle branch of the printed pressure lacks the r^2 of the
  (25/2) term; continuity at r = 0.2 (value 5.5) and r = 0.4 (value
  3 + 4 ln 2) fixes it as 9 - 4 ln 0.2 + (25/2) r^2 - 20 r + 4 ln r.  The
  domain is [-1/2, 1/2]^2 with a quadrilateral mesh.  Amplitude A scales
  the velocity and background pressure P gives p = P + A^2 (p_G - (3 + 4 ln 2)),
  which keeps the steady balance dp/dr = rho v_phi^2 / r.
* Taylor-Green: amplitude A scales the velocity and A^2 the pressure
  perturbation.
* Sedov: the delta source is modelled by giving every thermodynamic dof of
  the element at the origin the value E / (rho0 |K|), so that the total
  internal energy equals E.
* Triple point (Sec. 6.1.4): density, pressure and adiabatic index are
  piecewise constant over three regions of [0,7] x [0,3] (x [0,1.5]).  The
  material of an element (its rho0, gamma and initial pressure) is the one
  at the element's centre, so rho0 and gamma are constant per element and
  the thermodynamic dofs of an element share its pressure.  On meshes whose
  faces contain the interfaces x = 1 and y = 1.5 this is the printed data
  exactly; the interfaces' own points, which the paper assigns with <= and
  >, are never evaluated.  Every other problem has rho0 = 1 and one gamma.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .fe import Q1_NODES_1D, Mesh


@dataclass(frozen=True)
class Problem:
    name: str  # "taylor_green", "sedov", "gresho", "triple_point"
    mesh: Mesh
    gamma: float
    use_av: bool
    cfl: float  # alpha in eq. adaptive-timestep
    amp: float = 1.0  # TG / Gresho amplitude
    p_bg: float = 3.0 + 4.0 * np.log(2.0)  # Gresho background pressure
    energy: float = 0.25  # Sedov deposited energy


def triple_point_regions(X: np.ndarray):
    """(rho0, gamma, p0) of the triple-point problem at positions X (n, d), Sec. 6.1.4:
    rho0 = 1 where x <= 1 or y <= 1.5, else 1/8; p0 = 1 where x <= 1, else 0.1;
    gamma = 1.5 where x <= 1 or y > 1.5, else 1.4."""
    x, y = X[:, 0], X[:, 1]
    left = x <= 1.0
    top = y > 1.5
    rho = np.where(left | ~top, 1.0, 0.125)
    gamma = np.where(left | top, 1.5, 1.4)
    p = np.where(left, 1.0, 0.1)
    return rho, gamma, p


def element_centres(mesh: Mesh) -> np.ndarray:
    E = mesh.elem_coords()
    return np.array(mesh.lo, float)[None, :] + (E + 0.5) * mesh.h[None, :]


def element_material(prob: Problem):
    """Per-element (rho0, gamma): the triple point's regions at the element centres, else (1, prob.gamma)."""
    n = prob.mesh.n_elem
    if prob.name == "triple_point":
        rho, gamma, _ = triple_point_regions(element_centres(prob.mesh))
        return rho, gamma
    return np.ones(n), np.full(n, float(prob.gamma))


def thermo_coords(mesh: Mesh) -> np.ndarray:
    """(N_E, d) physical positions of the Q1 dofs at t = 0."""
    E = mesh.elem_coords()
    h = mesh.h
    d = mesh.dim
    nt = 2 ** d
    loc = np.array([[(j >> c) & 1 for c in range(d)] for j in range(nt)])
    out = np.zeros((mesh.n_elem, nt, d))
    for c in range(d):
        out[:, :, c] = mesh.lo[c] + h[c] * (E[:, c][:, None] + Q1_NODES_1D[loc[:, c]][None, :])
    return out.reshape(-1, d)


def _velocity(prob: Problem, X: np.ndarray) -> np.ndarray:
    d = prob.mesh.dim
    pi = np.pi
    A = prob.amp
    if prob.name == "taylor_green":
        if d == 2:
            x, y = X[:, 0], X[:, 1]
            return A * np.stack([np.sin(pi * x) * np.cos(pi * y), -np.cos(pi * x) * np.sin(pi * y)], axis=1)
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        return A * np.stack([np.sin(pi * x) * np.cos(pi * y) * np.cos(pi * z),
                             -np.cos(pi * x) * np.sin(pi * y) * np.cos(pi * z),
                             np.zeros_like(x)], axis=1)
    if prob.name == "gresho":
        x, y = X[:, 0], X[:, 1]
        r = np.hypot(x, y)
        vphi = np.where(r < 0.2, 5.0 * r, np.where(r < 0.4, 2.0 - 5.0 * r, 0.0))
        rs = np.where(r > 0, r, 1.0)
        return A * np.stack([-vphi * y / rs, vphi * x / rs], axis=1)
    if prob.name in ("sedov", "triple_point"):
        return np.zeros_like(X)
    raise ValueError(prob.name)


def gresho_pressure_profile(r: np.ndarray) -> np.ndarray:
    """p_G(r) of the Gresho vortex (with the r^2 reading of the middle branch)."""
    r = np.asarray(r, dtype=np.float64)
    rs = np.where(r > 0, r, 1.0)
    mid = 9.0 - 4.0 * np.log(0.2) + 12.5 * r * r - 20.0 * r + 4.0 * np.log(rs)
    return np.where(r < 0.2, 5.0 + 12.5 * r * r, np.where(r < 0.4, mid, 3.0 + 4.0 * np.log(2.0)))


def _pressure(prob: Problem, X: np.ndarray) -> np.ndarray:
    d = prob.mesh.dim
    pi = np.pi
    A = prob.amp
    if prob.name == "taylor_green":
        if d == 2:
            x, y = X[:, 0], X[:, 1]
            return 1.0 + A * A * (np.cos(2 * pi * x) + np.cos(2 * pi * y)) / 4.0
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        return 100.0 + A * A * ((np.cos(2 * pi * x) + np.cos(2 * pi * y)) * (np.cos(2 * pi * z) + 2.0) - 2.0) / 16.0
    if prob.name == "gresho":
        r = np.hypot(X[:, 0], X[:, 1])
        return prob.p_bg + A * A * (gresho_pressure_profile(r) - (3.0 + 4.0 * np.log(2.0)))
    raise ValueError(prob.name)


def initial_state(prob: Problem):
    """Return (x0, v0, e0): positions and velocities (N_V), energies (N_E)."""
    mesh = prob.mesh
    d = mesh.dim
    X = mesh.node_coords()
    x0 = X.T.reshape(-1).copy()  # component-major
    v0 = _velocity(prob, X).T.reshape(-1).copy()
    rho0 = 1.0
    if prob.name == "triple_point":
        rho, gamma, p = triple_point_regions(element_centres(mesh))
        e0 = np.repeat(p / ((gamma - 1.0) * rho), 2 ** d)
    elif prob.name == "sedov":
        e0 = np.zeros(mesh.NE)
        vol = float(np.prod(mesh.h))
        e0[: 2 ** d] = prob.energy / (rho0 * vol)  # element 0 touches the origin
    else:
        Xt = thermo_coords(mesh)
        e0 = _pressure(prob, Xt) / ((prob.gamma - 1.0) * rho0)
    return x0, v0, e0
