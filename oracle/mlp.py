"""MLP surrogate of the reduced force coefficients (oracle, test infrastructure).

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path imports this module.

The paper has no learned component (it mentions neural-network ROMs only as
related work, Sec. 1); the surrogate is an addition to the hyper-reduced ROM
of Sec. 3.3 and the windowed SNS system (eq. rom-hr-sns):

* Network: z0 = ([x^, v^, e^, t] - mu_in) / s_in; for l = 1..L-1,
  a_l = tanh(r(a_{l-1}) r(W_l) + b_l); output y~ = r(a_{L-1}) r(W_L) + b_L and
  y = mu_out + s_out * y~.  r() rounds an operand to bfloat16 (round to
  nearest even); every product is accumulated exactly here (FP64), in FP32 on
  the GPU.  W_l is stored (fan_in x fan_out), row-major.
* Output: [F^1 (n_v), f (n_e), H (n_e x n_v, row-major)] at the state y^ =
  (x^, v^, e^), with f the energy right-hand side at the state's own velocity,
  so that for a contraction velocity v^_c the energy right-hand side is
  F^tv(v^_c) = f + H (v^_c - v^).  This is exact for the DEIM chain because
  F^T v_c is linear in v_c (eq. forceOneforceTv) and v~_c = v_os + Phi_v v^_c;
  H only multiplies the O(dt) difference v^_c - v^, whereas f is the physical
  quantity itself (a split into F^T v_os and H v^ would be a small difference
  of large terms wherever the flow is nearly divergence free).
* Loss: mean over the batch and the outputs of (y~ - t~)^2 with the targets
  normalised by the same mu_out, s_out.
* Backward: delta_L = 2 (y~ - t~) / (B d_out); grad W_l = r(a_{l-1})^T r(delta_l);
  grad b_l = sum over the batch of delta_l; delta_{l-1} =
  (r(delta_l) r(W_l)^T) * (1 - a_{l-1}^2).
* Adam with bias correction on FP32 master weights (here FP64).

The surrogate ROM (``run_surrogate``) replaces the sampled lift, force and
projection by the network between audits: the first step of every window
with a network and then every K-th accepted step is an audit step, taken with
the DEIM chain exactly as the plain ROM (``rom.rom_step``); it also supplies
the time-step estimate tau used by the step control until the next audit, and
compares the network's F^1 and F^tv (at the audit's first stage) with the
DEIM chain's (``audit``).  A discrepancy above ``tol`` switches the window to
the DEIM chain for the rest of the window (fallback).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fom as F
from . import rom as R


# ----------------------------------------------------------------- bfloat16

def bf16(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) and return as float64.

    A value is first rounded to float32 (round to nearest), then the low 16
    bits of its float32 pattern are rounded away: add 0x7FFF plus the lowest
    kept bit and truncate.  NaN stays NaN, infinities stay infinite.
    """
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


def identity(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)


# ------------------------------------------------------------------ network

@dataclass
class MLP:
    W: list  # (fan_in, fan_out) per layer
    b: list
    mu_in: np.ndarray
    s_in: np.ndarray
    mu_out: np.ndarray
    s_out: np.ndarray

    @property
    def sizes(self):
        return [self.W[0].shape[0]] + [w.shape[1] for w in self.W]


def glorot_init(sizes, g: np.random.Generator):
    """Uniform Glorot initial weights and zero biases, drawn from the given generator."""
    W, b = [], []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (fi + fo))
        W.append(g.uniform(-lim, lim, (fi, fo)))
        b.append(np.zeros(fo))
    return W, b


def normalisation(X: np.ndarray):
    """Column means and standard deviations (population); a zero deviation is replaced by 1."""
    mu = X.mean(axis=0)
    s = X.std(axis=0)
    s = np.where(s > 0, s, 1.0)
    return mu, s


def forward(net: MLP, X: np.ndarray, r=bf16):
    """Activations [z0, a_1, ..., a_{L-1}, y~] for raw inputs X (B x d_in)."""
    acts = [(np.asarray(X, dtype=np.float64) - net.mu_in) / net.s_in]
    L = len(net.W)
    for l in range(L):
        z = r(acts[-1]) @ r(net.W[l]) + net.b[l]
        acts.append(np.tanh(z) if l < L - 1 else z)
    return acts


def predict(net: MLP, X: np.ndarray, r=bf16) -> np.ndarray:
    return net.mu_out + net.s_out * forward(net, X, r)[-1]


def loss(net: MLP, X: np.ndarray, T: np.ndarray, r=bf16) -> float:
    yt = forward(net, X, r)[-1]
    tt = (np.asarray(T, dtype=np.float64) - net.mu_out) / net.s_out
    return float(np.mean((yt - tt) ** 2))


def backward(net: MLP, X: np.ndarray, T: np.ndarray, r=bf16):
    """Gradients (gW list, gb list) of ``loss`` with respect to W and b."""
    acts = forward(net, X, r)
    B, dout = acts[-1].shape
    tt = (np.asarray(T, dtype=np.float64) - net.mu_out) / net.s_out
    delta = 2.0 * (acts[-1] - tt) / (B * dout)
    L = len(net.W)
    gW, gb = [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        gW[l] = r(acts[l]).T @ r(delta)
        gb[l] = delta.sum(axis=0)
        if l > 0:
            delta = (r(delta) @ r(net.W[l]).T) * (1.0 - acts[l] ** 2)
    return gW, gb


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: list = field(default_factory=list)
    v: list = field(default_factory=list)

    def step(self, params: list, grads: list):
        """One update of every array in params (in place)."""
        if not self.m:
            self.m = [np.zeros_like(p) for p in params]
            self.v = [np.zeros_like(p) for p in params]
        self.t += 1
        c1 = 1.0 - self.beta1 ** self.t
        c2 = 1.0 - self.beta2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.beta1
            m += (1.0 - self.beta1) * g
            v *= self.beta2
            v += (1.0 - self.beta2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


# ------------------------------------------------------ surrogate of the ROM

def layout(win: R.WindowROM):
    nx, nv, ne = win.dims
    return nx + nv + ne + 1, nv + ne + ne * nv


def net_input(yhat, t) -> np.ndarray:
    return np.concatenate([yhat[0], yhat[1], yhat[2], [t]])


def split_output(win: R.WindowROM, y: np.ndarray):
    _, nv, ne = win.dims
    return y[:nv], y[nv:nv + ne], y[nv + ne:].reshape(ne, nv)


def deim_targets(op: F.Operator, win: R.WindowROM, yhat) -> np.ndarray:
    """[F^1, f, H] of the DEIM chain at the lifted state of yhat (eq. rom-hr-sns).

    F^1 = A1 (F.1)_Z1 at y~ = y_os + Phi y^ on the sampled elements;
    f = A2 (F^T v~)_Z2 with v~ = v_os + Phi_v v^ and column k of H is A2 (F^T Phi_v e_k)_Z2.
    """
    NV, NE = op.mesh.NV, op.mesh.NE
    els = win.elems
    st = F.stress(op, R.lift_rows(win, 0, yhat[0], win.rows_k, NV), R.lift_rows(win, 1, yhat[1], win.rows_k, NV),
                  R.lift_rows(win, 2, yhat[2], win.rows_t, NE), elems=els)
    f1 = win.A1 @ F.force_one(op, st, elems=els)[win.Z1]
    nv = win.dims[1]
    f = win.A2 @ F.force_tv(op, st, R.lift_rows(win, 1, yhat[1], win.rows_k, NV), elems=els)[win.Z2]
    H = np.zeros((win.dims[2], nv))
    for k in range(nv):
        u = np.zeros(NV)
        u[win.rows_k] = win.Phi[1][win.rows_k, k]
        H[:, k] = win.A2 @ F.force_tv(op, st, u, elems=els)[win.Z2]
    return np.concatenate([f1, f, H.ravel()])


def training_set(op: F.Operator, rom: R.ROM, w: int, trajs: list, windows_of_snap: list):
    """Inputs and targets from FOM snapshots projected onto window w's bases.

    trajs: oracle trajectories; windows_of_snap[k][j] is the window of snapshot j of trajectory k.
    Snapshot j of a trajectory is its state j (stage and step states in order, times from
    ``snapshot_times``).
    """
    win = rom.windows[w]
    X, T = [], []
    for tr, wins in zip(trajs, windows_of_snap):
        times = snapshot_times(tr)
        for j, (x, v, e) in enumerate(tr.snaps):
            if wins[j] != w:
                continue
            yh = tuple(win.Phi[f].T @ (s - win.os[f]) for f, s in enumerate((x, v, e)))
            X.append(net_input(yh, times[j]))
            T.append(deim_targets(op, win, yh))
    return np.array(X), np.array(T)


def snapshot_times(tr) -> list:
    """Times of the recorded states: stage n+1/2 at t_n + dt_n/2, step n+1 at t_{n+1}."""
    out = []
    for n, h in enumerate(tr.dt):
        out.append(tr.t[n] + 0.5 * h)
        out.append(tr.t[n + 1])
    return out


@dataclass
class SurrogateRun:
    t: list
    dt: list
    w: int
    yhat: tuple
    rejections: int = 0
    audits: int = 0
    surrogate_steps: int = 0
    fallback_windows: list = field(default_factory=list)


def surrogate_step(win: R.WindowROM, net: MLP, xh, vh, eh, t, dt, r=bf16):
    """One RK2-average step with the network's reduced forces (eq. RK2-avg-rom-hr)."""
    f1, f, H = split_output(win, predict(net, net_input((xh, vh, eh), t)[None, :], r)[0])
    v_half = vh - 0.5 * dt * f1
    e_half = eh + 0.5 * dt * (f + H @ (v_half - vh))
    x_half = xh + 0.5 * dt * (win.bx + win.Bxv @ v_half)
    f1, f, H = split_output(win, predict(net, net_input((x_half, v_half, e_half), t + 0.5 * dt)[None, :], r)[0])
    v_new = vh - dt * f1
    v_bar = 0.5 * (vh + v_new)
    e_new = eh + dt * (f + H @ (v_bar - v_half))
    x_new = xh + dt * (win.bx + win.Bxv @ v_bar)
    return x_new, v_new, e_new


def audit(op: F.Operator, win: R.WindowROM, net: MLP, yhat, t, dt, r=bf16):
    """DEIM step plus the network's discrepancy at the first stage.

    Returns (new state, tau, discrepancy) with discrepancy = max(d1, d2):
    d1 = |F^1_net - F^1| / (|F^1| + |s_F1|) at y^_n and
    d2 = |F^tv_net - F^tv| / (|F^tv| + |s_f|) at the DEIM chain's midpoint velocity v^_{1/2},
    where s_F1 and s_f are the network's output scales (training standard deviations) of F^1 and
    f: they keep a locally small force (F^tv vanishes where the flow is divergence free) from
    turning an error that is small on the scale the network was trained on into a large relative one.
    """
    new, half, tau = R.rom_step(op, win, *yhat, dt)
    tgt = deim_targets(op, win, yhat)
    f1_d, f_d, H_d = split_output(win, tgt)
    f1_m, f_m, H_m = split_output(win, predict(net, net_input(yhat, t)[None, :], r)[0])
    v_half = half[1]
    ftv_d = f_d + H_d @ (v_half - yhat[1])
    ftv_m = f_m + H_m @ (v_half - yhat[1])
    nv, ne = win.dims[1], win.dims[2]
    s_f1 = np.linalg.norm(net.s_out[:nv]) if net is not None else 0.0
    s_f = np.linalg.norm(net.s_out[nv:nv + ne]) if net is not None else 0.0

    def rel(a, b, scale):
        return np.linalg.norm(a - b) / scale if scale > 0 else np.linalg.norm(a - b)

    d1 = rel(f1_m, f1_d, np.linalg.norm(f1_d) + s_f1)
    d2 = rel(ftv_m, ftv_d, np.linalg.norm(ftv_d) + s_f)
    return new, tau, max(d1, d2)


def run_surrogate(op: F.Operator, rom: R.ROM, nets: dict, y0: tuple, t_final: float, audit_every: int,
                  tol: float, r=bf16, max_steps=10**7, fixed_dt=None) -> SurrogateRun:
    """Online phase with the network in the windows of ``nets`` ({window: MLP}), DEIM elsewhere.

    The first step of a window and every audit_every-th accepted step after it is an audit; a failed
    audit, or a surrogate step whose new state is not finite, sends the rest of the window to DEIM
    (the non-finite step itself is redone with DEIM).  With ``fixed_dt`` every step has that size and
    nothing is rejected (as ``rom.run_rom``).
    """
    w = 0
    yhat = R.initial_coords(rom, y0)
    t = 0.0
    run = SurrogateRun([0.0], [], 0, yhat)
    win = rom.windows[0]
    st = F.stress(op, R.lift_rows(win, 0, yhat[0], win.rows_k, op.mesh.NV),
                  R.lift_rows(win, 1, yhat[1], win.rows_k, op.mesh.NV),
                  R.lift_rows(win, 2, yhat[2], win.rows_t, op.mesh.NE), elems=win.elems)
    dt = F.BETA1 * float(np.min(st.tau)) if fixed_dt is None else fixed_dt
    since = 0  # accepted steps since the last audit in this window
    fallen = False
    tau_est = np.inf
    n = 0
    while F.not_done(t, t_final) and n < max_steps:
        h = fixed_dt if fixed_dt is not None else F.final_step_clip(t, t_final, dt)
        net = nets.get(w)
        win = rom.windows[w]
        if net is None or fallen:
            new, _, tau = R.rom_step(op, win, *yhat, h)
        elif since % audit_every == 0:
            new, tau, disc = audit(op, win, net, yhat, t, h, r)
            run.audits += 1
            tau_est = tau
            if not disc <= tol:
                fallen = True
                run.fallback_windows.append(w)
        else:
            new = surrogate_step(win, net, *yhat, t, h, r)
            tau = tau_est
            if not all(np.all(np.isfinite(c)) for c in new):
                # a non-finite network state: the rest of the window, this step included, takes DEIM
                fallen = True
                run.fallback_windows.append(w)
                new, _, tau = R.rom_step(op, win, *yhat, h)
        if fixed_dt is None:
            if h >= tau:
                dt = F.BETA1 * h
                run.rejections += 1
                continue
            dt = F.BETA2 * h if h <= F.GAMMA_DT * tau else h
        if net is not None and not fallen and since % audit_every != 0:
            run.surrogate_steps += 1
        yhat = new
        t = t + h
        n += 1
        since += 1
        run.t.append(t)
        run.dt.append(h)
        while w + 1 < len(rom.windows) and R.reached(t, rom.windows[w].T_end):
            w += 1
            yhat = R.switch_window(rom, w, yhat)
            since = 0
            fallen = False
            tau_est = np.inf
    run.w = w
    run.yhat = yhat
    return run
