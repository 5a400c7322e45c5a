"""Full-order model: force, mass matrices and RK2-average (oracle, test infrastructure).

Semi-discrete system (eq. fom): M_V dv/dt = -F.1, M_E de/dt = F^T.v,
dx/dt = v, with F the N_V x N_E force matrix of the current state.  The paper
defers the definition of F and of the artificial viscosity to Dobrev et al.;
this oracle uses the corner-force form

    F_{(a,c), j} = int_{Omega(t)} (sigma : grad(N_a e_c)) phi_j dx,

so that, with Jacobian J = dx/dxi of the moving map and the pulled-back
stress  sigma~_q = w_q det J_q sigma_q J_q^{-T}  at quadrature point q,

    (F.1)_{a,c}   = sum_q sum_i sigma~_q[c, i] dN_a/dxi_i(q)        (sum_j phi_j = 1)
    (F^T.u)_j     = sum_q phi_j(q) sum_{c,i} sigma~_q[c, i] (sum_a u_{a,c} dN_a/dxi_i(q)).

Stress: sigma = -p I + mu eps(v), p = (gamma-1) rho e (eq. EOS),
eps = sym grad v, rho_q = rho0 det J0 / det J (Lagrangian mass conservation);
rho0 and gamma are the element's (piecewise constant in the triple-point
problem, uniform otherwise).
Artificial viscosity (reading; the paper refers to Dobrev Sec. 6):

    mu = rho l^2 q2 max(0, -lambda_min(eps)) + rho l q1 c_s psi0,
    psi0 = max(0, -tr eps) / (|eps|_F + 1e-8 c_s / l + 1e-300),
    l = h_min = sigma_min(J) / k,   c_s = sqrt(max(gamma (gamma-1) e, 0)),
    q1 = 1/2, q2 = 2.

Time-step estimate (eq. adaptive-timestep):
tau_q = alpha / (c_s / h_min + alpha_mu mu / (rho h_min^2)), alpha_mu = 2.5.

Boundary conditions v.n = 0 are imposed by elimination: constrained rows of
F.1 are zeroed and the kinematic mass matrix has identity rows/columns there.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fe import ORDER, Mesh, ref_tables
from .problems import Problem, element_material, initial_state

ALPHA_MU = 2.5
BETA1 = 0.85
BETA2 = 1.02
GAMMA_DT = 0.8
AV_Q1 = 0.5
AV_Q2 = 2.0


class TangledMesh(RuntimeError):
    pass


@dataclass
class Operator:
    """Everything about the semi-discretisation that is fixed in time."""

    prob: Problem
    mesh: Mesh
    ref: object
    en: np.ndarray  # (E, nk) element -> global node
    et: np.ndarray  # (E, nt) element -> thermo dof
    cq: np.ndarray  # (E, nq) rho0 det J0 w_q
    gamma_e: np.ndarray  # (E,) adiabatic index of each element
    Mv_scalar: sp.csr_matrix  # scalar Q2 mass matrix
    Mv: sp.csr_matrix  # d copies (component-major), no elimination
    Mv_eff: sp.csc_matrix  # eliminated
    Me: sp.csr_matrix  # block-diagonal thermodynamic mass
    constrained: np.ndarray
    _lu: object = field(default=None, repr=False)
    _me_inv: np.ndarray = field(default=None, repr=False)

    def solve_v(self, rhs: np.ndarray) -> np.ndarray:
        if self._lu is None:  # factorised on first use (force-only uses of large meshes skip it)
            self._lu = spla.splu(self.Mv_eff)
        r = np.where(self.constrained, 0.0, rhs)
        return self._lu.solve(r)

    def solve_e(self, rhs: np.ndarray) -> np.ndarray:
        nt = self.et.shape[1]
        return np.einsum("kij,kj->ki", self._me_inv, rhs.reshape(-1, nt)).reshape(-1)


def _element_geometry(op_ref, en, x, n_nodes, d):
    """J[E, q, c, i] = sum_a x_{a,c} dN_a/dxi_i(q)."""
    xe = np.stack([x[c * n_nodes + en] for c in range(d)], axis=2)  # (E, nk, d)
    return np.einsum("eac,qai->eqci", xe, op_ref.dB)


def build_operator(prob: Problem) -> Operator:
    mesh = prob.mesh
    d = mesh.dim
    ref = ref_tables(d)
    en = mesh.elem_nodes()
    et = mesh.elem_thermo()
    x0, _, _ = initial_state(prob)
    J0 = _element_geometry(ref, en, x0, mesh.n_nodes, d)
    det0 = np.linalg.det(J0)
    rho0, gamma_e = element_material(prob)
    cq = rho0[:, None] * det0 * ref.w[None, :]
    # scalar kinematic mass: sum_q cq N_a N_b
    Mloc = np.einsum("eq,qa,qb->eab", cq, ref.B, ref.B)
    nk = en.shape[1]
    rows = np.repeat(en, nk, axis=1).ravel()
    cols = np.tile(en, (1, nk)).ravel()
    Ms = sp.coo_matrix((Mloc.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    Mv = sp.block_diag([Ms] * d, format="csr")
    constrained = mesh.constrained_dofs()
    keep = sp.diags((~constrained).astype(float))
    Mv_eff = (keep @ Mv @ keep + sp.diags(constrained.astype(float))).tocsc()
    # thermodynamic mass: block diagonal, sum_q cq phi_i phi_j
    Meloc = np.einsum("eq,qi,qj->eij", cq, ref.Bt, ref.Bt)
    Me = sp.block_diag(list(Meloc), format="csr")
    op = Operator(prob, mesh, ref, en, et, cq, gamma_e, Ms, Mv, Mv_eff, Me, constrained)
    op._me_inv = np.linalg.inv(Meloc)
    return op


@dataclass
class Stress:
    """Per-quadrature-point quantities of one force evaluation."""

    sig_t: np.ndarray  # (E, nq, d, d) pulled-back stress sigma~
    tau: np.ndarray  # (E, nq) time-step estimate
    det: np.ndarray  # (E, nq)
    rho: np.ndarray  # (E, nq)


def stress(op: Operator, x, v, e, elems=None) -> Stress:
    """Pulled-back stress at every quadrature point of the listed elements."""
    prob = op.prob
    mesh = op.mesh
    d = mesh.dim
    ref = op.ref
    en = op.en if elems is None else op.en[elems]
    et = op.et if elems is None else op.et[elems]
    cq = op.cq if elems is None else op.cq[elems]
    nn = mesh.n_nodes
    J = _element_geometry(ref, en, x, nn, d)
    det = np.linalg.det(J)
    if np.any(det <= 0.0):
        raise TangledMesh("det J <= 0 at some quadrature point")
    Jinv = np.linalg.inv(J)
    w = ref.w[None, :]
    rho = cq / (w * det)
    eq = np.einsum("ej,qj->eq", e[et], ref.Bt)
    g = (op.gamma_e if elems is None else op.gamma_e[elems])[:, None]
    p = (g - 1.0) * rho * eq
    cs = np.sqrt(np.maximum(g * (g - 1.0) * eq, 0.0))
    hmin = np.linalg.svd(J, compute_uv=False)[..., -1] / ORDER
    I = np.eye(d)
    sig = -p[..., None, None] * I
    mu = np.zeros_like(p)
    if prob.use_av:
        G = _element_geometry(ref, en, v, nn, d)
        gradv = G @ Jinv  # d v_c / d x_k
        eps = 0.5 * (gradv + np.swapaxes(gradv, -1, -2))
        lam_min = np.linalg.eigvalsh(eps)[..., 0]
        tr = np.trace(eps, axis1=-2, axis2=-1)
        nrm = np.sqrt(np.sum(eps * eps, axis=(-2, -1)))
        ell = hmin
        psi0 = np.maximum(0.0, -tr) / (nrm + 1e-8 * cs / ell + 1e-300)
        mu = rho * ell * ell * AV_Q2 * np.maximum(0.0, -lam_min) + rho * ell * AV_Q1 * cs * psi0
        sig = sig + mu[..., None, None] * eps
    sig_t = (w * det)[..., None, None] * (sig @ np.swapaxes(Jinv, -1, -2))
    denom = cs / hmin + ALPHA_MU * mu / (rho * hmin * hmin)
    with np.errstate(divide="ignore"):
        tau = np.where(denom > 0.0, prob.cfl / np.where(denom > 0, denom, 1.0), np.inf)
    return Stress(sig_t, tau, det, rho)


def force_one(op: Operator, st: Stress, elems=None, eliminate=True) -> np.ndarray:
    """F.1 assembled over the listed elements (all by default)."""
    mesh = op.mesh
    d = mesh.dim
    en = op.en if elems is None else op.en[elems]
    loc = np.einsum("eqci,qai->eac", st.sig_t, op.ref.dB)  # (E, nk, d)
    out = np.zeros(mesh.NV)
    for c in range(d):
        np.add.at(out, c * mesh.n_nodes + en, loc[:, :, c])
    if eliminate:
        out[op.constrained] = 0.0
    return out


def force_tv(op: Operator, st: Stress, u: np.ndarray, elems=None) -> np.ndarray:
    """F^T.u on the thermodynamic dofs of the listed elements (others zero)."""
    mesh = op.mesh
    d = mesh.dim
    en = op.en if elems is None else op.en[elems]
    et = op.et if elems is None else op.et[elems]
    Gu = _element_geometry(op.ref, en, u, mesh.n_nodes, d)  # sum_a u_{a,c} dN_a/dxi_i
    s = np.einsum("eqci,eqci->eq", st.sig_t, Gu)
    loc = np.einsum("eq,qj->ej", s, op.ref.Bt)
    out = np.zeros(mesh.NE)
    out[et.ravel()] = loc.ravel()
    return out


def total_energy(op: Operator, v, e) -> float:
    """Discrete total energy 1/2 v^T M_V v + 1^T M_E e."""
    return 0.5 * float(v @ (op.Mv @ v)) + float(np.ones_like(e) @ (op.Me @ e))


@dataclass
class StepResult:
    x: np.ndarray
    v: np.ndarray
    e: np.ndarray
    xh: np.ndarray
    vh: np.ndarray
    eh: np.ndarray
    tau: float
    stages: list = field(default_factory=list)  # every stage state the force was evaluated at, after y_n


def rk2avg_step(op: Operator, x, v, e, dt) -> StepResult:
    """One RK2-average step (eq. RK2-avg): stage state n+1/2, then n+1."""
    s1 = stress(op, x, v, e)
    vh = v - 0.5 * dt * op.solve_v(force_one(op, s1))
    eh = e + 0.5 * dt * op.solve_e(force_tv(op, s1, vh))
    xh = x + 0.5 * dt * vh
    s2 = stress(op, xh, vh, eh)
    vn = v - dt * op.solve_v(force_one(op, s2))
    vbar = 0.5 * (v + vn)
    en_ = e + dt * op.solve_e(force_tv(op, s2, vbar))
    xn = x + dt * vbar
    tau = min(float(np.min(s1.tau)), float(np.min(s2.tau)))
    return StepResult(xn, vn, en_, xh, vh, eh, tau)


def rhs(op: Operator, x, v, e):
    """Right-hand side of eq. fom at one state, (dx/dt, dv/dt, de/dt) = (v, -M_V^{-1} F.1, M_E^{-1} F^T.v),
    the force contracted with the state's own velocity; and the state's step estimate."""
    st = stress(op, x, v, e)
    return (v, -op.solve_v(force_one(op, st)), op.solve_e(force_tv(op, st, v))), float(np.min(st.tau))


def rk4_step(op: Operator, x, v, e, dt) -> StepResult:
    """One classical RK4 step (eq. RK4, eq. RK4coeff) of the whole state y = (x, v, e):
    k1 = f(y), k2 = f(y + dt/2 k1), k3 = f(y + dt/2 k2), k4 = f(y + dt k3),
    y_{n+1} = y + dt/6 (k1 + 2 k2 + 2 k3 + k4).  tau is the minimum over the four stages.  The
    returned stage state (xh, vh, eh) is y + dt/2 k1, the half-step state of the first stage, and
    ``stages`` holds the three stage states y + dt/2 k1, y + dt/2 k2, y + dt k3."""
    y = (x, v, e)
    k1, t1 = rhs(op, *y)
    y2 = tuple(a + 0.5 * dt * k for a, k in zip(y, k1))
    k2, t2 = rhs(op, *y2)
    y3 = tuple(a + 0.5 * dt * k for a, k in zip(y, k2))
    k3, t3 = rhs(op, *y3)
    y4 = tuple(a + dt * k for a, k in zip(y, k3))
    k4, t4 = rhs(op, *y4)
    yn = tuple(a + dt / 6.0 * (p + 2.0 * q + 2.0 * r + s) for a, p, q, r, s in zip(y, k1, k2, k3, k4))
    return StepResult(yn[0], yn[1], yn[2], y2[0], y2[1], y2[2], min(t1, t2, t3, t4), [y2, y3, y4])


def final_step_clip(t, t_final, dt):
    """Step size actually attempted: dt, or the remainder when it (nearly) fits."""
    rem = t_final - t
    return rem if rem <= dt * (1.0 + 1e-9) else dt


def not_done(t, t_final):
    return t_final - t > 1e-12 * t_final


@dataclass
class Trajectory:
    t: list  # accepted times t_0 .. t_Nt
    dt: list  # accepted step sizes
    x: np.ndarray  # final state
    v: np.ndarray
    e: np.ndarray
    snap_t: list = field(default_factory=list)
    snaps: list = field(default_factory=list)  # (x, v, e) at stage and step states
    snap_kind: list = field(default_factory=list)  # 0 = stage n+1/2, 1 = step n+1
    snap_step: list = field(default_factory=list)  # step index n+1 the snapshot belongs to
    r: int = 2  # snapshots per accepted step: its stage states, then its step state
    rejections: int = 0
    energy: list = field(default_factory=list)


def run_fom(op: Operator, t_final: float, fixed_dt=None, dt_replay=None, record=True,
            max_steps=10**7, scheme="rk2avg") -> Trajectory:
    """Integrate the FOM from t = 0 to t_final with RK2-average (eq. RK2-avg) or, with scheme="rk4",
    classical RK4 (eq. RK4).  Snapshots of every accepted step are the stage states its forces were
    evaluated at after y_n, then the step state: r = 2 per step for RK2-average (y_{n+1/2}, y_{n+1}),
    r = 4 for RK4 (y_n + h/2 k1, y_n + h/2 k2, y_n + h k3, y_{n+1}), so that every stage increment
    lies in the snapshots' span.

    Step control (Sec. 2.2.3): attempt h = min(dt, t_final - t); if h >= tau
    (tau = min over the quadrature points of all stages) reject and retry
    with dt = beta1 h; otherwise accept and, if h <= gamma tau, grow the next
    step to beta2 h.  The first dt is beta1 tau(y_0).  With ``fixed_dt`` no
    step is rejected; with ``dt_replay`` the given step sizes are used.
    """
    if scheme not in ("rk2avg", "rk4"):
        raise ValueError(scheme)
    step = rk4_step if scheme == "rk4" else rk2avg_step
    x, v, e = initial_state(op.prob)
    t = 0.0
    tr = Trajectory([0.0], [], x, v, e, r=4 if scheme == "rk4" else 2)
    tr.energy.append(total_energy(op, v, e))
    if fixed_dt is not None:
        dt = fixed_dt
    elif dt_replay is None:
        dt = BETA1 * float(np.min(stress(op, x, v, e).tau))
    n = 0
    while (not_done(t, t_final) if dt_replay is None else n < len(dt_replay)) and n < max_steps:
        h = dt_replay[n] if dt_replay is not None else final_step_clip(t, t_final, dt)
        r = step(op, x, v, e, h)
        if fixed_dt is None and dt_replay is None:
            if h >= r.tau:
                dt = BETA1 * h
                tr.rejections += 1
                continue
            dt = BETA2 * h if h <= GAMMA_DT * r.tau else h
        if record:
            if scheme == "rk4":
                tr.snap_t += [t + 0.5 * h, t + 0.5 * h, t + h, t + h]
                tr.snaps += [*r.stages, (r.x, r.v, r.e)]
                tr.snap_kind += [0, 0, 0, 1]
                tr.snap_step += [n + 1] * 4
            else:
                tr.snap_t += [t + 0.5 * h, t + h]
                tr.snaps += [(r.xh, r.vh, r.eh), (r.x, r.v, r.e)]
                tr.snap_kind += [0, 1]
                tr.snap_step += [n + 1, n + 1]
        x, v, e = r.x, r.v, r.e
        t = t + h
        n += 1
        tr.t.append(t)
        tr.dt.append(h)
        tr.energy.append(total_energy(op, v, e))
    tr.x, tr.v, tr.e = x, v, e
    return tr
