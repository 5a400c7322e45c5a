"""Hyper-reduced SNS ROM with RK2-average and time windows (oracle, test infrastructure).

Online system (eq. rom-hr-sns, windowed as eq. rom-hr-tw):

    dv^/dt = -F^1,  de^/dt = F^tv,  dx^/dt = Phi_x^T v_os + Phi_x^T Phi_v v^,

where, with the SNS bases Phi_F1 = M_V Phi_v and Phi_Ftv = M_E Phi_e
(Sec. 3.6), the reduced right-hand sides are the DEIM least-squares
coefficients F^1 = (Z1^T Phi_F1)^+ Z1^T F.1 and F^tv = (Z2^T Phi_Ftv)^+ Z2^T F^T.v
(eq. sol-ls-hyper, eq. sol-ls-hyper-2).  The fully discrete scheme is
RK2-average applied to it (eq. RK2-avg-rom-hr): the energy uses the lifted
midpoint velocity in the first stage and the lifted average velocity in the
second.  The FOM state is lifted only at the dofs of the sampled elements
(y~ = y_os + Phi y^, eq. discretesolrepresentation) and the step size comes
from the same controller as the FOM, evaluated on the lifted state at the
sampled elements' quadrature points.

On entering window w (once t >= T_w up to a relative 1e-12, see ``reached``)
the reduced coordinates are re-expressed in the new basis by lifting with the
old one and projecting (eq. ic-tw):
y^w = Phi_w^T (y_os^{w-1} + Phi_{w-1} y^{w-1} - y_os^w).

The relative error at the final time is the Euclidean one of eq. relerrors.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from . import deim as D
from . import fom as F
from .pod import pod_basis
from .windows import snapshot_matrices, window_start_states


@dataclass
class WindowROM:
    T_end: float
    Phi: list  # [Phi_x, Phi_v, Phi_e]
    os: list  # [x_os, v_os, e_os]
    Z1: np.ndarray
    Z2: np.ndarray
    A1: np.ndarray
    A2: np.ndarray
    elems: np.ndarray
    rows_k: np.ndarray  # kinematic dofs touched by the sampled elements
    rows_t: np.ndarray  # thermodynamic dofs of the sampled elements
    Bxv: np.ndarray
    bx: np.ndarray
    sigma: list = field(default_factory=list)
    trans: list = field(default_factory=list)  # [(T, c)] per field from the previous window

    @property
    def dims(self):
        return tuple(P.shape[1] for P in self.Phi)


@dataclass
class ROM:
    windows: list
    init_mass: list = field(default_factory=lambda: [None, None, None])  # per field: M of the initial projection
    train_offsets: list = field(default_factory=list)  # [window][trajectory] (x, v, e) snapshot offsets


def sns_bases(op: F.Operator, Phi_v: np.ndarray, Phi_e: np.ndarray):
    """Phi_F1 = M_V Phi_v (eliminated form), Phi_Ftv = M_E Phi_e (Sec. 3.6)."""
    return op.Mv_eff @ Phi_v, op.Me @ Phi_e


def sampled_rows(op: F.Operator, elems: np.ndarray):
    mesh = op.mesh
    nodes = np.unique(op.en[elems].ravel())
    rows_k = np.concatenate([c * mesh.n_nodes + nodes for c in range(mesh.dim)])
    rows_t = op.et[elems].ravel()
    return np.sort(rows_k), np.sort(rows_t)


SAMPLERS = {"deim": D.greedy_deim, "qdeim": D.qdeim}


def build_window(op, S_list, os_list, T_end, energy_frac, n_fixed, lam, n_max=0, sampler="deim",
                 basis="euclidean") -> WindowROM:
    Phis, sigmas = [], []
    for f in range(3):
        nf = n_fixed[f] if n_fixed else 0
        Phi, sigma, _ = pod_basis(S_list[f], energy_frac, nf, n_max)
        Phis.append(Phi)
        sigmas.append(sigma)
    if basis == "mass":  # velocity and energy bases orthonormal in M_V and M_E
        Phis[1] = mass_orthonormal(Phis[1], op.Mv_eff)
        Phis[2] = mass_orthonormal(Phis[2], op.Me)
    PF1, PFtv = sns_bases(op, Phis[1], Phis[2])
    nv, ne = Phis[1].shape[1], Phis[2].shape[1]
    pick = SAMPLERS[sampler]
    Z1 = pick(PF1, int(round(lam[0] * nv)))
    Z2 = pick(PFtv, int(round(lam[1] * ne)))
    A1 = D.deim_pinv(PF1, Z1)
    A2 = D.deim_pinv(PFtv, Z2)
    elems = D.closure_elements(op.mesh, op.en, Z1, Z2)
    rows_k, rows_t = sampled_rows(op, elems)
    Bxv = Phis[0].T @ Phis[1]
    bx = Phis[0].T @ os_list[1]
    return WindowROM(T_end, Phis, list(os_list), Z1, Z2, A1, A2, elems, rows_k, rows_t, Bxv, bx, sigmas)


def window_transition(Phi_new, os_new, Phi_old, os_old, M=None):
    """Reduced initial condition of a window from the previous window's coordinates,
    yhat_new = T yhat_old + c.  M None: orthogonal projection of the lifted state os_old + Phi_old
    yhat_old onto the new window (eq. ic-tw).  M given: the projection oblique in the M inner product,
    T = Mhat^{-1} Phi_new^T M Phi_old, c = Mhat^{-1} Phi_new^T M (os_old - os_new), Mhat = Phi_new^T M
    Phi_new (eq. ic2-tw), which minimises the M-norm of the error of the lifted initial state."""
    if M is None:
        return Phi_new.T @ Phi_old, Phi_new.T @ (os_old - os_new)
    MP = M @ Phi_new
    Mhat = Phi_new.T @ MP
    return np.linalg.solve(Mhat, MP.T @ Phi_old), np.linalg.solve(Mhat, MP.T @ (os_old - os_new))


def mass_orthonormal(Phi: np.ndarray, M) -> np.ndarray:
    """The same subspace in a basis orthonormal in the M inner product (Sec. 3.2, eq. rmass: the alternative
    with reduced mass matrix Phi^T M Phi = I): Phi L^{-T}, L the Cholesky factor of Phi^T M Phi."""
    L = np.linalg.cholesky(Phi.T @ (M @ Phi))
    return np.linalg.solve(L, Phi.T).T


def idw_weights(params, mu, r: float = 2.0) -> np.ndarray:
    """Inverse distance weights of eq. interpolate_os: w_k = d(mu, mu_k)^-r / sum_j d(mu, mu_j)^-r with
    the Euclidean distance, or the unit weight of the first training parameter at distance 0."""
    P = np.atleast_2d(np.asarray(params, dtype=np.float64).reshape(len(params), -1))
    d = np.linalg.norm(P - np.asarray(mu, dtype=np.float64).reshape(1, -1), axis=1)
    w = np.zeros(len(d))
    zero = np.nonzero(d == 0.0)[0]
    if len(zero):
        w[zero[0]] = 1.0
        return w
    w = d ** (-r)
    return w / np.sum(w)


def interpolated_offsets(train_offsets: list, params, mu, r: float = 2.0) -> list:
    """eq. interpolate_os for every window: train_offsets[w][k] is the offset (x, v, e) of window w
    at training parameter k; returns one (x, v, e) per window for the parameter mu."""
    w = idw_weights(params, mu, r)
    return [tuple(sum(wk * np.asarray(o[f]) for wk, o in zip(w, per_k)) for f in range(3)) for per_k in train_offsets]


def build_rom(op, trajs, offsets, T_ends, energy_frac=0.9999, n_fixed=None, lam=(2.0, 2.0),
              n_max=0, online_offsets=None, sampler="deim", window_ic="orthogonal",
              window_offsets="initial", basis="euclidean") -> ROM:
    """Offline phase: per-window POD, SNS, DEIM (greedy, or Q-DEIM with sampler="qdeim") and
    reduced operators.  window_ic: "orthogonal" (eq. ic-tw) or "oblique" (eq. ic2-tw: velocity and
    energy projected in the M_V and M_E inner products, position as in eq. ic-tw).

    window_offsets (Sec. 4.6): "initial", every window's snapshots relative to offsets (one initial
    state per trajectory); "window_start", window w's snapshots of trajectory k relative to that
    trajectory's state at the window's start.  online_offsets: one (x, v, e) for every window, or a
    list with one per window (for instance the interpolated offsets of eq. interpolate_os).
    The training offsets per window and trajectory are kept in ROM.train_offsets.

    basis="mass": the velocity and energy bases of every window are made orthonormal in M_V and M_E
    (same subspaces, reduced mass matrices I); the projections of the initial state and of the
    window changes are then taken in those inner products (so window_ic must be "oblique")."""
    if window_ic not in ("orthogonal", "oblique"):
        raise ValueError(window_ic)
    if basis not in ("euclidean", "mass") or (basis == "mass" and window_ic != "oblique"):
        raise ValueError("basis must be 'euclidean', or 'mass' with window_ic='oblique'")
    if window_offsets == "initial":
        by_window = [list(offsets)] * len(T_ends)
    elif window_offsets == "window_start":
        starts = [window_start_states(tr, y0, T_ends) for tr, y0 in zip(trajs, offsets)]
        by_window = [[starts[k][w] for k in range(len(trajs))] for w in range(len(T_ends))]
    else:
        raise ValueError(window_offsets)
    mats = snapshot_matrices(trajs, offsets, T_ends, offsets_by_window=by_window)
    os_on = offsets[0] if online_offsets is None else online_offsets
    per_window_os = isinstance(os_on, list)
    wins = []
    for w, Tw in enumerate(T_ends):
        win = build_window(op, mats[w], os_on[w] if per_window_os else os_on, Tw, energy_frac, n_fixed, lam, n_max,
                           sampler, basis)
        if w > 0:
            prev = wins[-1]
            mass = [None, op.Mv_eff, op.Me] if window_ic == "oblique" else [None, None, None]
            win.trans = [window_transition(win.Phi[f], win.os[f], prev.Phi[f], prev.os[f], mass[f]) for f in range(3)]
        wins.append(win)
    rom = ROM(wins)
    rom.train_offsets = by_window
    if basis == "mass":
        rom.init_mass = [None, op.Mv_eff, op.Me]
    return rom


def lift_rows(win: WindowROM, f: int, yhat: np.ndarray, rows: np.ndarray, N: int) -> np.ndarray:
    """Full-size vector holding os + Phi yhat on ``rows`` (zero elsewhere)."""
    out = np.zeros(N)
    out[rows] = win.os[f][rows] + win.Phi[f][rows, :] @ yhat
    return out


def lift_full(win: WindowROM, f: int, yhat: np.ndarray) -> np.ndarray:
    return win.os[f] + win.Phi[f] @ yhat


@dataclass
class ROMStage:
    xh: np.ndarray
    vh: np.ndarray
    eh: np.ndarray


def rom_step(op: F.Operator, win: WindowROM, xh, vh, eh, dt):
    """One RK2-average step of the hyper-reduced SNS system; returns new coords and tau."""
    mesh = op.mesh
    NV, NE = mesh.NV, mesh.NE
    els = win.elems

    def lift_state(xc, vc, ec):
        return (lift_rows(win, 0, xc, win.rows_k, NV), lift_rows(win, 1, vc, win.rows_k, NV),
                lift_rows(win, 2, ec, win.rows_t, NE))

    def f1_hat(st):
        return win.A1 @ F.force_one(op, st, elems=els)[win.Z1]

    def ftv_hat(st, vc_hat):
        u = lift_rows(win, 1, vc_hat, win.rows_k, NV)
        return win.A2 @ F.force_tv(op, st, u, elems=els)[win.Z2]

    # stage 1 at y~_n
    s1 = F.stress(op, *lift_state(xh, vh, eh), elems=els)
    v_half = vh - 0.5 * dt * f1_hat(s1)
    e_half = eh + 0.5 * dt * ftv_hat(s1, v_half)
    x_half = xh + 0.5 * dt * (win.bx + win.Bxv @ v_half)
    # stage 2 at y~_{n+1/2}
    s2 = F.stress(op, *lift_state(x_half, v_half, e_half), elems=els)
    v_new = vh - dt * f1_hat(s2)
    v_bar = 0.5 * (vh + v_new)
    e_new = eh + dt * ftv_hat(s2, v_bar)
    x_new = xh + dt * (win.bx + win.Bxv @ v_bar)
    tau = min(float(np.min(s1.tau)), float(np.min(s2.tau)))
    return (x_new, v_new, e_new), (x_half, v_half, e_half), tau


def rom_step_rk4(op: F.Operator, win: WindowROM, xh, vh, eh, dt):
    """One classical RK4 step (eq. RK4) of the hyper-reduced SNS system of a window:
    d x^/dt = b_x + B_xv v^, d v^/dt = -F^1(y~), d e^/dt = F^tv(y~; v~), with y~ the lifted state
    and the force contracted with the state's own lifted velocity.  Returns new coords, the
    first stage's half-step coords and tau (the minimum over the four stages)."""
    mesh = op.mesh
    NV, NE = mesh.NV, mesh.NE
    els = win.elems

    def f(xc, vc, ec):
        lifted = (lift_rows(win, 0, xc, win.rows_k, NV), lift_rows(win, 1, vc, win.rows_k, NV),
                  lift_rows(win, 2, ec, win.rows_t, NE))
        st = F.stress(op, *lifted, elems=els)
        k = (win.bx + win.Bxv @ vc, -(win.A1 @ F.force_one(op, st, elems=els)[win.Z1]),
             win.A2 @ F.force_tv(op, st, lifted[1], elems=els)[win.Z2])
        return k, float(np.min(st.tau))

    y = (xh, vh, eh)
    k1, t1 = f(*y)
    y2 = tuple(a + 0.5 * dt * k for a, k in zip(y, k1))
    k2, t2 = f(*y2)
    y3 = tuple(a + 0.5 * dt * k for a, k in zip(y, k2))
    k3, t3 = f(*y3)
    y4 = tuple(a + dt * k for a, k in zip(y, k3))
    k4, t4 = f(*y4)
    yn = tuple(a + dt / 6.0 * (p + 2.0 * q + 2.0 * r + s) for a, p, q, r, s in zip(y, k1, k2, k3, k4))
    return yn, y2, min(t1, t2, t3, t4)


@dataclass
class ROMRun:
    t: list
    dt: list
    w: int
    yhat: tuple
    rejections: int = 0
    window_of_step: list = field(default_factory=list)
    os: tuple = None  # offsets in use at the end (offsets="previous" changes them at every switch)
    energy: list = field(default_factory=list)  # total energy of the lifted state at t_0 and every accepted step


@dataclass
class EnergyOps:
    """Reduced form of the discrete total energy of a window's lifted state.

    RK2-average conserves E = 1/2 v^T M_V v + 1^T M_E e of the semi-discrete system (Sec. 2.2.1).
    For v = v_os + Phi_v v^ and e = e_os + Phi_e e^ it is a quadratic in the reduced coordinates,
    with the reduced mass matrix Mhat_V = Phi_v^T M_V Phi_v of eq. rmass (Sec. 3.2):

        E = c + m_v^T v^ + 1/2 v^T Mhat_V v^ + m_e^T e^,
        m_v = Phi_v^T M_V v_os,  m_e = Phi_e^T M_E 1,  c = 1/2 v_os^T M_V v_os + 1^T M_E e_os.

    M_V is the kinematic mass matrix without boundary elimination, the one of the FOM's total energy."""

    Mv_hat: np.ndarray
    mv: np.ndarray
    me: np.ndarray
    c: float


def energy_ops(op: F.Operator, win: WindowROM) -> EnergyOps:
    Pv, Pe = win.Phi[1], win.Phi[2]
    vos, eos = np.asarray(win.os[1]), np.asarray(win.os[2])
    MPv = op.Mv @ Pv
    Mvos = op.Mv @ vos
    Me1 = op.Me.T @ np.ones(op.mesh.NE)
    c = 0.5 * float(vos @ Mvos) + float(Me1 @ eos)
    return EnergyOps(Pv.T @ MPv, Pv.T @ Mvos, Pe.T @ Me1, c)


def reduced_energy(ops: EnergyOps, vh: np.ndarray, eh: np.ndarray) -> float:
    return ops.c + float(ops.mv @ vh) + 0.5 * float(vh @ (ops.Mv_hat @ vh)) + float(ops.me @ eh)


def initial_coords(rom: ROM, y0: tuple):
    """Coordinates of the initial state in the first window: its orthogonal projection, or with a
    mass inner product the M-orthogonal one, (Phi^T M Phi)^{-1} Phi^T M (y0 - os)."""
    win = rom.windows[0]
    out = []
    for f in range(3):
        d = y0[f] - win.os[f]
        M = rom.init_mass[f]
        if M is None:
            out.append(win.Phi[f].T @ d)
        else:
            MP = M @ win.Phi[f]
            out.append(np.linalg.solve(win.Phi[f].T @ MP, MP.T @ d))
    return tuple(out)


def switch_window(rom: ROM, w: int, yhat: tuple) -> tuple:
    win = rom.windows[w]
    return tuple(win.trans[f][0] @ yhat[f] + win.trans[f][1] for f in range(3))


SWITCH_RTOL = 1e-12


def reached(t: float, T_end: float) -> bool:
    """Whether the online time t has reached the window end T_end.

    Windows chosen by number of snapshots end at FOM step times, which a ROM
    that reproduces the FOM's step sizes meets up to rounding; t within
    SWITCH_RTOL relative below T_end counts as reaching it, so that the switch
    does not depend on the last bits of the accumulated time.
    """
    return t >= T_end * (1.0 - SWITCH_RTOL)


def with_offsets(win: WindowROM, os: tuple) -> WindowROM:
    """The window with other offsets: its offset-dependent operator b_x = Phi_x^T v_os follows."""
    return replace(win, os=[np.asarray(o) for o in os], bx=win.Phi[0].T @ np.asarray(os[1]))


def run_rom(op: F.Operator, rom: ROM, y0: tuple, t_final: float, dt_replay=None, fixed_dt=None,
            max_steps=10**7, offsets="given", scheme="rk2avg") -> ROMRun:
    """Online phase from t = 0 to t_final (same step control as the FOM), with RK2-average
    (eq. RK2-avg-rom-hr) or, with scheme="rk4", classical RK4 (eq. RK4) of the reduced system.

    offsets="given": every window uses the offsets it was built with and the reduced state moves to
    the next window by eq. ic-tw (or ic2-tw).  offsets="previous" (eq. previous_os): the first window
    uses its own offsets; at each switch the ROM's state lifted with the closing window becomes the
    next window's offset, so the reduced state restarts at zero.  run.os holds the offsets in use at
    the end."""
    if offsets not in ("given", "previous"):
        raise ValueError(offsets)
    if scheme not in ("rk2avg", "rk4"):
        raise ValueError(scheme)
    step = rom_step_rk4 if scheme == "rk4" else rom_step
    w = 0
    yhat = initial_coords(rom, y0)
    t = 0.0
    run = ROMRun([0.0], [], 0, yhat)
    cur = rom.windows[0]
    eops = {}

    def energy_of(win, y):
        if id(win) not in eops:
            eops[id(win)] = (win, energy_ops(op, win))  # keep win alive so its id stays unique
        return reduced_energy(eops[id(win)][1], y[1], y[2])

    run.energy.append(energy_of(cur, yhat))
    if fixed_dt is not None:
        dt = fixed_dt
    elif dt_replay is None:
        win = rom.windows[0]
        st = F.stress(op, lift_rows(win, 0, yhat[0], win.rows_k, op.mesh.NV),
                      lift_rows(win, 1, yhat[1], win.rows_k, op.mesh.NV),
                      lift_rows(win, 2, yhat[2], win.rows_t, op.mesh.NE), elems=win.elems)
        dt = F.BETA1 * float(np.min(st.tau))
    n = 0
    while (F.not_done(t, t_final) if dt_replay is None else n < len(dt_replay)) and n < max_steps:
        h = dt_replay[n] if dt_replay is not None else F.final_step_clip(t, t_final, dt)
        new, _, tau = step(op, cur, *yhat, h)
        if fixed_dt is None and dt_replay is None:
            if h >= tau:
                dt = F.BETA1 * h
                run.rejections += 1
                continue
            dt = F.BETA2 * h if h <= F.GAMMA_DT * tau else h
        yhat = new
        t = t + h
        n += 1
        run.t.append(t)
        run.dt.append(h)
        run.window_of_step.append(w)
        while w + 1 < len(rom.windows) and reached(t, rom.windows[w].T_end):
            w += 1
            if offsets == "previous":
                lifted = tuple(lift_full(cur, f, yhat[f]) for f in range(3))
                cur = with_offsets(rom.windows[w], lifted)
                yhat = tuple(np.zeros(n) for n in cur.dims)
            else:
                yhat = switch_window(rom, w, yhat)
                cur = rom.windows[w]
        run.energy.append(energy_of(cur, yhat))
    run.w = w
    run.yhat = yhat
    run.os = tuple(np.asarray(o) for o in cur.os)
    return run


def final_lift(rom: ROM, run: ROMRun):
    win = rom.windows[run.w]
    os = getattr(run, "os", None)
    if os is not None:
        win = replace(win, os=list(os))
    return tuple(lift_full(win, f, run.yhat[f]) for f in range(3))


def relative_errors(fom_final: tuple, rom_final: tuple):
    """Per-field ||y - y~||_2 / ||y||_2 at the final time (eq. relerrors), order (x, v, e)."""
    return tuple(float(np.linalg.norm(a - b) / np.linalg.norm(a)) for a, b in zip(fom_final, rom_final))
