"""Further pins of the oracle: closed-form artificial viscosity, the step controller's branches,
the sampled-element closure under partial sampling, 3D Taylor-Green consistency and the reduced
total energy (CPU)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import deim as D
from oracle import fom as F
from oracle import rom as R
from oracle.fe import Mesh
from oracle.problems import Problem, initial_state
from oracle.windows import snapshot_matrices
from tests.oracle_adapter import oracle_problem


# ------------------------------------------------------------ artificial viscosity

@pytest.mark.parametrize("dim,rates", [(2, (0.7, 1.9)), (3, (0.7, 1.9, -0.4)), (3, (1.3, 0.2, 0.5))],
                         ids=["2d", "3d-mixed", "3d-compressed"])
def test_viscosity_closed_form_under_homogeneous_motion(dim, rates):
    """Mesh scaled by s, v = -diag(a) x: every quantity of the stress has a closed form.

    With x = s X on an n^d mesh of the unit box: J = s h I, rho = s^-d, l = h_min = s h / 2,
    eps = -diag(a), lambda_min(eps) = -max a, tr eps = -sum a, |eps|_F = |a|_2; the viscosity is
    mu = rho l^2 q2 max(0, max a) + rho l q1 c_s psi0 with psi0 = max(0, sum a) / (|a|_2 + 1e-8 c_s / l),
    sigma = -p I - mu diag(a), sigma~ = w det J sigma / (s h), tau = alpha / (c_s / l + 2.5 mu / (rho l^2)).
    Swapping q1 and q2, l for l^2, the eigenvalue picked, the trace or the norm changes the values."""
    n, s, e0, gam, alpha = 3, 0.9, 2.0, 1.4, 0.5
    a = np.array(rates, dtype=float)
    mesh = Mesh(dim, (n,) * dim, (0.0,) * dim, (1.0,) * dim)
    op = F.build_operator(Problem("sedov", mesh, gam, True, alpha))
    X = mesh.node_coords().T  # (d, nn)
    x = s * X
    v = -a[:, None] * x
    e = np.full(mesh.NE, e0)
    st = F.stress(op, x.ravel(), v.ravel(), e)
    h = 1.0 / n
    rho = s ** (-dim)
    ell = s * h / 2.0
    cs = np.sqrt(gam * (gam - 1.0) * e0)
    p = (gam - 1.0) * rho * e0
    psi0 = max(0.0, a.sum()) / (np.sqrt(np.sum(a * a)) + 1e-8 * cs / ell + 1e-300)
    mu = rho * ell * ell * 2.0 * max(0.0, a.max()) + rho * ell * 0.5 * cs * psi0
    sig = -p * np.eye(dim) - mu * np.diag(a)
    detJ = (s * h) ** dim
    want = op.ref.w[:, None, None] * detJ * sig[None] / (s * h)
    np.testing.assert_allclose(st.rho, rho, rtol=1e-14)
    np.testing.assert_allclose(st.sig_t, np.broadcast_to(want, st.sig_t.shape), rtol=1e-13, atol=1e-14 * np.abs(want).max())
    tau = alpha / (cs / ell + 2.5 * mu / (rho * ell * ell))
    np.testing.assert_allclose(st.tau, tau, rtol=1e-14)
    assert mu > 0.0


# ------------------------------------------------------------ step controller

# Hand-derived run of the controller of Sec. 2.2.3 (beta1 = 0.85, beta2 = 1.02, gamma = 0.8) to
# t_final = 1.3 with tau(y_0) = 0.4, so the first attempt is 0.85 * 0.4 = 0.34.  Each attempt is
# followed by the step estimate the scripted solver returns ("h" means exactly the attempted step):
#   0.34        tau 0.3   -> 0.34 >= 0.3 rejected, next 0.85 * 0.34 = 0.289
#   0.289       tau 0.5   -> accepted (t = 0.289), 0.289 <= 0.4 grows to 1.02 * 0.289 = 0.29478
#   0.29478     tau h     -> equal to tau: rejected, next 0.85 * 0.29478 = 0.250563
#   0.250563    tau 0.3   -> accepted (t = 0.539563), 0.250563 > 0.24: kept
#   0.250563    tau 0.32  -> accepted (t = 0.790126), 0.250563 <= 0.256 grows to 0.25557426
#   0.25557426  tau 1.0   -> accepted (t = 1.04570026), grows to 0.2606857452
#   the remainder 1.3 - 1.04570026 = 0.25429974 is attempted; tau 1.0 -> accepted, t = 1.3
T_FINAL = 1.3
SCRIPT = [0.3, 0.5, "h", 0.3, 0.32, 1.0, 1.0]
ATTEMPTS = [0.34, 0.289, 0.29478, 0.250563, 0.250563, 0.25557426, 0.25429974]
ACCEPTED = [0.289, 0.250563, 0.250563, 0.25557426, 0.25429974]


class _Scripted:
    def __init__(self):
        self.k = 0
        self.attempts = []

    def tau(self, h):
        t = SCRIPT[self.k]
        self.k += 1
        self.attempts.append(h)
        return h if t == "h" else t


class _Tau:
    def __init__(self, tau):
        self.tau = np.array([tau])


def test_fom_step_controller_follows_the_hand_derived_sequence(monkeypatch):
    op = F.build_operator(oracle_problem(W.tg2d(2)))
    sc = _Scripted()

    def fake_step(op_, x, v, e, dt):
        return F.StepResult(x, v, e, x, v, e, sc.tau(dt))

    monkeypatch.setattr(F, "stress", lambda *a, **k: _Tau(0.4))
    monkeypatch.setattr(F, "rk2avg_step", fake_step)
    tr = F.run_fom(op, T_FINAL, record=False)
    np.testing.assert_allclose(sc.attempts, ATTEMPTS, rtol=1e-14)
    np.testing.assert_allclose(tr.dt, ACCEPTED, rtol=1e-14)
    assert tr.rejections == 2 and len(tr.dt) == 5
    assert abs(tr.t[-1] - T_FINAL) <= 1e-15


def test_rom_step_controller_follows_the_hand_derived_sequence(monkeypatch):
    op = F.build_operator(oracle_problem(W.tg2d(2)))
    NV, NE = op.mesh.NV, op.mesh.NE
    z = [np.zeros((NV, 1)), np.zeros((NV, 1)), np.zeros((NE, 1))]
    os_ = [np.zeros(NV), np.zeros(NV), np.zeros(NE)]
    e1 = np.array([0])
    win = R.WindowROM(T_FINAL, z, os_, e1, e1, np.zeros((1, 1)), np.zeros((1, 1)), e1, np.arange(NV), np.arange(NE),
                      np.zeros((1, 1)), np.zeros(1))
    rom = R.ROM([win])
    sc = _Scripted()

    def fake_rom_step(op_, win_, xh, vh, eh, dt):
        return (xh, vh, eh), (xh, vh, eh), sc.tau(dt)

    monkeypatch.setattr(F, "stress", lambda *a, **k: _Tau(0.4))
    monkeypatch.setattr(R, "rom_step", fake_rom_step)
    run = R.run_rom(op, rom, tuple(os_), T_FINAL)
    np.testing.assert_allclose(sc.attempts, ATTEMPTS, rtol=1e-14)
    np.testing.assert_allclose(run.dt, ACCEPTED, rtol=1e-14)
    assert run.rejections == 2


# ------------------------------------------------------------ closure of the sampled rows

def test_closure_under_partial_sampling_is_the_hand_listed_elements():
    """3 x 3 mesh (7 x 7 nodes, node id gx + 7 gy, element ex + 3 ey).

    Kinematic rows: x of vertex (2, 2) -> elements 0, 1, 3, 4; y of the mid-edge node (5, 0) on the
    bottom wall -> element 2 only; x of the centre node (3, 3) of element 4; x of the corner node
    (0, 6) -> element 6.  Thermodynamic rows: dof 3 of element 8, which touches no sampled node,
    and dof 0 of element 4."""
    mesh = Mesh(2, (3, 3), (0.0, 0.0), (1.0, 1.0))
    nn = mesh.n_nodes
    assert nn == 49
    Z1 = np.array([2 + 7 * 2, nn + 5, 3 + 7 * 3, 0 + 7 * 6])
    Z2 = np.array([8 * 4 + 3, 4 * 4 + 0])
    els = D.closure_elements(mesh, mesh.elem_nodes(), Z1, Z2)
    np.testing.assert_array_equal(els, [0, 1, 2, 3, 4, 6, 8])


# ------------------------------------------------------------ 3D Taylor-Green consistency

def test_consistency_taylor_green_3d_acceleration():
    """AV off, t = 0: -M_V^-1 F.1 -> -grad p = (pi/8)(sin 2pi x (cos 2pi z + 2), sin 2pi y (cos 2pi z + 2),
    (cos 2pi x + cos 2pi y) sin 2pi z) and M_E^-1 F^T v -> -p div v = 0, at second order."""
    errs_a, errs_e = [], []
    for n in (4, 8, 16):
        mesh = Mesh(3, (n, n, n), (0.0,) * 3, (1.0,) * 3)
        op = F.build_operator(Problem("taylor_green", mesh, 5 / 3, False, 0.1))
        x, v, e = initial_state(op.prob)
        st = F.stress(op, x, v, e)
        rhs = np.where(op.constrained, 0.0, -F.force_one(op, st))
        a, info = spla.cg(op.Mv_eff, rhs, rtol=1e-13, maxiter=2000)
        assert info == 0
        X = mesh.node_coords()
        px, py, pz = (2 * np.pi * X[:, c] for c in range(3))
        exact = np.pi / 8 * np.concatenate([np.sin(px) * (np.cos(pz) + 2), np.sin(py) * (np.cos(pz) + 2),
                                            (np.cos(px) + np.cos(py)) * np.sin(pz)])
        inside = np.all((X > 0) & (X < 1), axis=1)
        mask = ~op.constrained & np.tile(inside, 3)
        errs_a.append(np.abs(a - exact)[mask].max())
        errs_e.append(np.abs(op.solve_e(F.force_tv(op, st, v))).max())
    rate_a = np.log2(errs_a[0] / errs_a[1]), np.log2(errs_a[1] / errs_a[2])
    rate_e = np.log2(errs_e[0] / errs_e[1]), np.log2(errs_e[1] / errs_e[2])
    # the max-norm rate approaches 2 from below on these coarse meshes, as in 2D
    assert rate_a[0] > 1.0 and rate_a[1] > 1.7 and rate_a[1] > rate_a[0], (errs_a, rate_a)
    assert min(rate_e) > 1.8, (errs_e, rate_e)


# ------------------------------------------------------------ reduced total energy

@pytest.fixture(scope="module")
def tg_fom():
    wl = W.tg2d(8)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=wl.fixed_dt)
    return wl, op, tr, initial_state(op.prob)


@pytest.mark.parametrize("basis", ["euclidean", "mass"])
def test_reduced_energy_is_the_total_energy_of_the_lifted_state(tg_fom, basis):
    wl, op, tr, y0 = tg_fom
    win_ic = "oblique" if basis == "mass" else "orthogonal"
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(6, 6, 6), basis=basis, window_ic=win_ic)
    win = rom.windows[0]
    ops = R.energy_ops(op, win)
    if basis == "mass":  # eq. rmass with M-orthonormal bases: the reduced mass matrix is the identity
        np.testing.assert_allclose(ops.Mv_hat, np.eye(6), atol=1e-13)
    rng = np.random.default_rng(4)
    for _ in range(4):
        vh, eh = rng.normal(size=6), rng.normal(size=6)
        full = F.total_energy(op, R.lift_full(win, 1, vh), R.lift_full(win, 2, eh))
        assert abs(R.reduced_energy(ops, vh, eh) - full) <= 1e-13 * abs(full)


def test_reduced_energy_is_conserved_when_the_rom_retraces_the_fom(tg_fom):
    """Full-rank bases and full sampling: the ROM is the FOM, whose RK2-average step conserves the
    total energy (Sec. 2.2.1), so the reduced energy stays at its initial value."""
    wl, op, tr, y0 = tg_fom
    mats = snapshot_matrices([tr], [y0], [wl.t_final])[0]
    ranks = []
    for S in mats:
        s = np.linalg.svd(S, compute_uv=False)
        ranks.append(int(np.sum(s > 1e-11 * s[0])))
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=ranks, lam=(1e9, 1e9))
    run = R.run_rom(op, rom, y0, wl.t_final, dt_replay=tr.dt)
    E = np.array(run.energy)
    assert len(E) == len(tr.dt) + 1
    assert abs(E[0] - tr.energy[0]) <= 1e-14 * abs(tr.energy[0])
    assert np.abs(E - E[0]).max() <= 1e-11 * abs(E[0])
    # a hyper-reduced ROM on 6 modes does not conserve it exactly, but stays close
    rom6 = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(6, 6, 6), lam=wl.lam)
    run6 = R.run_rom(op, rom6, y0, wl.t_final, fixed_dt=wl.fixed_dt)
    drift = np.abs(np.array(run6.energy) - run6.energy[0]).max() / abs(run6.energy[0])
    assert 0.0 < drift < 1e-2
