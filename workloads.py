"""Seeded synthetic workload definitions shared by the tests, smoke() and bench.py.

This module holds only parameters and random draws: mesh sizes, domains,
physical constants, time horizons, window and basis settings and the
parameter samples of batched instances.  It contains none of the method's
arithmetic, so both the oracle and the GPU path can be fed from it without
sharing any computation.

The benchmark problems are the paper's analytic initial-value problems
(Sec. 6.1): there is no dataset behind them, only the mesh files of the
original code, which are uniform boxes and are generated here.  Random
parameters come from NumPy's PCG64 seeded with 210411404; instance i takes
the i-th draw of each listed distribution, in the order listed.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

SEED = 210411404

TAYLOR_GREEN = "taylor_green"
SEDOV = "sedov"
GRESHO = "gresho"
TRIPLE_POINT = "triple_point"
PROBLEM_IDS = {TAYLOR_GREEN: 1, SEDOV: 2, GRESHO: 3, TRIPLE_POINT: 4}


@dataclass(frozen=True)
class Workload:
    name: str
    problem: str
    dim: int
    nel: tuple
    lo: tuple
    hi: tuple
    gamma: float
    use_av: bool
    cfl: float
    t_final: float
    fixed_dt: float = 0.0  # 0 = adaptive step control
    n_windows: int = 1
    window_mode: str = "samples"  # "samples" (by snapshot count) or "physical"
    energy_frac: float = 0.9999
    n_fixed: tuple = ()  # fixed POD dims (x, v, e); empty = energy criterion
    n_max: int = 0  # cap on POD dims (0 = none)
    lam: tuple = (2.0, 2.0)  # oversampling factors for F.1 and F^T.v
    amp: float = 1.0
    p_bg: float = 3.0 + 4.0 * np.log(2.0)
    energy: float = 0.25
    params: tuple = field(default_factory=tuple)  # per-instance dicts for batches

    @property
    def n_nodes(self) -> int:
        return int(np.prod([2 * n + 1 for n in self.nel[: self.dim]]))

    @property
    def NV(self) -> int:
        return self.dim * self.n_nodes

    @property
    def NE(self) -> int:
        return (2 ** self.dim) * int(np.prod(self.nel[: self.dim]))

    @property
    def n_elem(self) -> int:
        return int(np.prod(self.nel[: self.dim]))


def tg2d(n: int = 8) -> Workload:
    """2D Taylor-Green on [0,1]^2, fixed dt = 1e-3 to t = 0.1, one window, dims 6/6/6."""
    return Workload("tg2d", TAYLOR_GREEN, 2, (n, n), (0.0, 0.0), (1.0, 1.0), 5.0 / 3.0, True, 0.5, 0.1,
                    fixed_dt=1e-3, n_windows=1, n_fixed=(6, 6, 6))


def sedov2d(n: int = 64, t_final: float = 0.8, n_windows: int = 10, lam: tuple = (6.0, 6.0)) -> Workload:
    """2D Sedov blast on [0,1.2]^2, energy 0.25 in the origin element, adaptive dt.

    Oversampling lambda = 6 for both force components: at 32 x 32 and 64 x 64
    with 10 windows, lambda = 2 leaves the hyper-reduced ROM unstable (the
    shock front runs through unsampled elements and the mesh tangles); 6 is the
    value the paper uses for its long-time Sedov run (Table of long-time
    results).
    """
    return Workload("sedov2d", SEDOV, 2, (n, n), (0.0, 0.0), (1.2, 1.2), 1.4, True, 0.5, t_final,
                    n_windows=n_windows, window_mode="samples", energy=0.25, lam=tuple(lam))


def gresho2d(n: int = 48, t_final: float = 0.1) -> Workload:
    """2D Gresho vortex on [-1/2,1/2]^2, no artificial viscosity."""
    return Workload("gresho2d", GRESHO, 2, (n, n), (-0.5, -0.5), (0.5, 0.5), 5.0 / 3.0, False, 0.5, t_final)


def tg3d(n: int = 24, t_final: float = 0.05) -> Workload:
    return Workload("tg3d", TAYLOR_GREEN, 3, (n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 5.0 / 3.0, True, 0.1,
                    t_final, n_fixed=(20, 20, 20))


def sedov3d(n: int = 32, t_final: float = 0.8) -> Workload:
    return Workload("sedov3d", SEDOV, 3, (n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 1.4, True, 0.5, t_final,
                    n_windows=20, energy=0.25)


def triple_point(nel: tuple = (28, 12, 4), t_final: float = 0.8) -> Workload:
    """Triple point (Sec. 6.1.4) on [0,7] x [0,3] x [0,1.5] (2D: [0,7] x [0,3]), walls everywhere,
    v = 0, piecewise density, pressure and adiabatic index; artificial viscosity on, CFL 0.5.

    The default mesh, 28 x 12 x 4, is the size of the paper's table of FOM sizes (N_V = 38475,
    N_E = 10752); nel must put the interfaces x = 1 and y = 1.5 on element faces (nel_x a multiple
    of 7, nel_y even).  gamma here is unused: each element takes its region's."""
    dim = len(nel)
    hi = (7.0, 3.0, 1.5)[:dim]
    return Workload("triple_point", TRIPLE_POINT, dim, tuple(nel), (0.0,) * dim, hi, 1.5, True,
                    0.5, t_final)


def tg2d_param(n: int = 32, t_final: float = 0.2, n_inst: int = 64, seed: int = SEED) -> Workload:
    """Parametric 2D Taylor-Green: amplitude A ~ U[0.8, 1.2] per instance, training at 0.8, 1.0, 1.2.

    Fixed dt = 1e-3, one window, dims 20/20/20, lambda = 2; bases shared by every instance with the
    nominal (A = 1) initial state as offset, so the reduced initial state carries the amplitude.
    """
    amps = rng(seed).uniform(0.8, 1.2, n_inst)
    return Workload("tg2d_param", TAYLOR_GREEN, 2, (n, n), (0.0, 0.0), (1.0, 1.0), 5.0 / 3.0, True, 0.5, t_final,
                    fixed_dt=1e-3, n_windows=1, n_fixed=(20, 20, 20), params=tuple(dict(amp=float(a)) for a in amps))


def tg3d_param(n: int = 24, t_final: float = 0.05, n_inst: int = 64, seed: int = SEED, use_av: bool = False,
               n_fixed: tuple = (10, 10, 10)) -> Workload:
    """Parametric 3D Taylor-Green on [0,1]^3: amplitude A ~ U[0.8, 1.2] per instance (the draws of
    tg2d_param), training at 0.8, 1.0, 1.2; alpha = 0.1, the paper's Taylor-Green CFL.

    Fixed dt = 1.5625e-4 to t = 0.05 (320 steps), about the step estimate of the initial state at
    24^3 (1.57e-4 with alpha = 0.1); the FOM stays untangled with up to 2.5e-4 at A = 0.8 and 1.2.
    One window, dims 10/10/10, lambda = 2; bases shared by every instance with the nominal (A = 1)
    initial state as offset.  Artificial viscosity is off by default: with it on, the viscosity of
    this smooth flow (traceless strain, so a negative smallest eigenvalue everywhere) leaves the
    plain DEIM ROM at a few 1e-2 in v even at the training amplitudes, so no form reaches the 1e-3
    error at which the surrogate and DEIM forms are compared; without it the DEIM ROM is at 1e-5.
    """
    amps = rng(seed).uniform(0.8, 1.2, n_inst)
    return Workload("tg3d_param", TAYLOR_GREEN, 3, (n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 5.0 / 3.0, use_av,
                    0.1, t_final, fixed_dt=1.5625e-4, n_windows=1, n_fixed=tuple(n_fixed),
                    params=tuple(dict(amp=float(a)) for a in amps))


def sedov3d_param(n: int = 32, n_inst: int = 64, seed: int = SEED, lam: tuple = (6.0, 6.0)) -> Workload:
    """Parametric 3D Sedov blast on [0,1]^3: deposited energy E ~ U[0.2, 0.3] per instance, training
    at E = 0.2, 0.25, 0.3; adaptive dt (alpha = 0.5) to t = 0.8.

    20 windows by snapshot count over the training set, POD dims by the 0.9999 criterion (at most
    64), bases shared by every instance with the nominal (E = 0.25) initial state as offset, so the
    reduced initial state carries the energy.
    """
    energies = rng(seed).uniform(0.2, 0.3, n_inst)
    return Workload("sedov3d_param", SEDOV, 3, (n, n, n), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 1.4, True, 0.5, 0.8,
                    n_windows=20, energy=0.25, lam=tuple(lam), params=tuple(dict(energy=float(E)) for E in energies))


SEDOV_TRAIN_ENERGIES = (0.2, 0.25, 0.3)  # training energies of the parametric Sedov problem

TG_TRAIN_AMPS = (0.8, 1.0, 1.2)  # training amplitudes of the parametric Taylor-Green problems


def rng(seed: int = SEED) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gresho_batch(n_inst: int = 256, n: int = 48, t_final: float = 0.1, seed: int = SEED,
                 lam: tuple = (8.0, 8.0)) -> Workload:
    """Batched Gresho instances: A ~ U[0.5,1.5], P ~ U[3,7], dims ~ U{8..40}, windows ~ U{1..8}.

    Oversampling lambda = 8, the paper's value for its short-time Gresho ROM (Table of short-time
    results): with lambda = 2 or 4 about one instance in seven tangles its mesh at 48 x 48, mostly
    those with one or two windows.
    """
    g = rng(seed)
    amps = g.uniform(0.5, 1.5, n_inst)
    pbgs = g.uniform(3.0, 7.0, n_inst)
    dims = g.integers(8, 41, n_inst)
    wins = g.integers(1, 9, n_inst)
    params = tuple(dict(amp=float(a), p_bg=float(p), n=int(d), n_windows=int(w))
                   for a, p, d, w in zip(amps, pbgs, dims, wins))
    return replace(gresho2d(n, t_final), name="gresho2d_batch", window_mode="physical", params=params,
                   lam=tuple(lam))


def sedov_energies(n_inst: int = 64, seed: int = SEED) -> np.ndarray:
    return rng(seed).uniform(0.2, 0.3, n_inst)


def random_state(wl: Workload, seed: int, scale: float = 0.02):
    """A smooth-ish perturbed state for single-call parity tests.

    Positions are the nodes displaced by a small random field (keeping every
    element valid), velocities and energies are random with the problem's
    magnitudes.  Returns (x, v, e, v_c) as float64 arrays in the solver's
    layouts (component-major kinematic, element-major thermodynamic).
    """
    g = rng(seed)
    d = wl.dim
    axes = [np.linspace(wl.lo[c], wl.hi[c], 2 * wl.nel[c] + 1) for c in range(d)]
    grids = np.meshgrid(*axes, indexing="ij")
    X = np.stack([gr.transpose(tuple(reversed(range(d)))).ravel() for gr in grids], axis=0)  # (d, nn)
    h = np.array([(wl.hi[c] - wl.lo[c]) / wl.nel[c] for c in range(d)])
    x = (X + scale * h[:, None] * g.uniform(-1, 1, X.shape)).ravel()
    v = g.normal(0.0, 1.0, d * X.shape[1])
    e = g.uniform(0.5, 2.0, wl.NE)
    vc = g.normal(0.0, 1.0, d * X.shape[1])
    return x, v, e, vc
