"""Pins of the oracle's triple-point problem (Sec. 6.1.4) and RK4 integrator (eq. RK4), CPU only.

Triple point: masses and internal energies of the three regions in closed form, the pressure jump
across x = 1 as the only force of the initial state (its face integrals written out with Simpson
weights), the step estimate of the fastest sound speed, and exact energy conservation of RK2-average
with per-element density and adiabatic index.  RK4: fourth-order self-convergence, the full-basis
full-sampling ROM retracing the RK4 FOM, and the RK4 ROM's own fourth order.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fom as F
from oracle import rom as R
from oracle.fe import Mesh
from oracle.problems import Problem, element_material, initial_state
from oracle.windows import snapshot_matrices
from tests.oracle_adapter import oracle_problem

# region (rho0, p0, gamma) and volume: x <= 1 | x > 1, y <= 1.5 | x > 1, y > 1.5
REGIONS_2D = [(1.0, 1.0, 1.5, 1.0 * 3.0), (1.0, 0.1, 1.4, 6.0 * 1.5), (0.125, 0.1, 1.5, 6.0 * 1.5)]


def _regions(dim):
    depth = 1.5 if dim == 3 else 1.0
    return [(r, p, g, vol * depth) for r, p, g, vol in REGIONS_2D]


@pytest.mark.parametrize("nel", [(14, 4), (7, 2, 1), (14, 4, 2)], ids=["2d", "3d_coarse", "3d"])
def test_triple_point_masses_and_internal_energy_are_the_regions_sums(nel):
    op = F.build_operator(oracle_problem(W.triple_point(nel)))
    x, v, e = initial_state(op.prob)
    reg = _regions(len(nel))
    mass = sum(r * vol for r, _, _, vol in reg)  # 13.125 in 2D, 19.6875 in 3D
    ie = sum(p * vol / (g - 1.0) for _, p, g, vol in reg)  # 10.05 in 2D, 15.075 in 3D
    ones = np.ones(op.mesh.n_nodes)
    assert abs(ones @ (op.Mv_scalar @ ones) - mass) <= 1e-13 * mass
    assert abs(np.ones(op.mesh.NE) @ (op.Me @ e) - ie) <= 1e-13 * ie
    assert np.all(v == 0.0)
    assert abs(F.total_energy(op, v, e) - ie) <= 1e-13 * ie


def test_triple_point_materials_at_known_points():
    prob = oracle_problem(W.triple_point((14, 4)))
    rho, gamma = element_material(prob)
    _, _, e = initial_state(prob)
    E = prob.mesh.elem_coords()
    h = prob.mesh.h

    def elem_at(px, py):
        return int(np.flatnonzero((E[:, 0] == int(px // h[0])) & (E[:, 1] == int(py // h[1])))[0])

    for (px, py), (r, g, ee) in {(0.5, 0.5): (1.0, 1.5, 2.0), (0.5, 2.5): (1.0, 1.5, 2.0),
                                 (3.0, 1.0): (1.0, 1.4, 0.25), (6.9, 0.1): (1.0, 1.4, 0.25),
                                 (3.0, 2.0): (0.125, 1.5, 1.6), (6.9, 2.9): (0.125, 1.5, 1.6)}.items():
        K = elem_at(px, py)
        assert rho[K] == r and gamma[K] == g
        np.testing.assert_allclose(e[4 * K:4 * K + 4], ee, rtol=1e-15)


@pytest.mark.parametrize("nel", [(14, 4), (14, 4, 2)], ids=["2d", "3d"])
def test_triple_point_initial_force_is_the_pressure_jump(nel):
    """v = 0, so sigma = -p I.  Integrating -p dN_a/dx_c by parts region by region leaves only the
    interface x = 1, where p jumps from 1 to 0.1: (F.1)_{a,x} = -(1 - 0.1) int_{x=1} N_a ds; every other
    entry is zero (p is constant across y = 1.5, and the walls' rows are eliminated).  The face
    integral of a Q2 shape function is a product of 1D Simpson weights: h/3 at an element vertex
    (summed over the two elements that share it), 2h/3 at an edge midpoint."""
    op = F.build_operator(oracle_problem(W.triple_point(nel)))
    x, v, e = initial_state(op.prob)
    F1 = F.force_one(op, F.stress(op, x, v, e))
    mesh = op.mesh
    X = mesh.node_coords()
    h = mesh.h
    d = mesh.dim
    nn = mesh.n_nodes
    expect = np.zeros(mesh.NV)
    on = np.isclose(X[:, 0], 1.0)
    w = np.ones(nn)
    for c in range(1, d):
        k = np.rint((X[:, c] - mesh.lo[c]) / (0.5 * h[c])).astype(int)  # half-spacing index along axis c
        top = 2 * mesh.nel[c]
        wc = np.where(k % 2 == 1, 2.0 * h[c] / 3.0, h[c] / 3.0)
        w *= np.where((k == 0) | (k == top), h[c] / 6.0, wc)
    expect[:nn] = np.where(on, -0.9 * w, 0.0)
    expect[op.constrained] = 0.0
    scale = np.abs(expect).max()
    assert np.abs(F1 - expect).max() <= 1e-13 * scale


def test_triple_point_step_estimate_is_set_by_the_fastest_sound_speed():
    """At rest mu = 0 and tau_q = alpha h_min / c_s with c_s^2 = gamma (gamma - 1) e = gamma p / rho:
    1.5, 0.14, 1.2 in the three regions, so the left region (c_s = sqrt 1.5) limits the step, with
    h_min = min(h) / 2."""
    wl = W.triple_point((14, 4, 2))
    op = F.build_operator(oracle_problem(wl))
    st = F.stress(op, *initial_state(op.prob))
    tau = float(np.min(st.tau))
    expect = wl.cfl * (min(op.mesh.h) / 2.0) / np.sqrt(1.5)
    assert abs(tau - expect) <= 1e-14 * expect


def test_triple_point_rk2avg_conserves_total_energy():
    """RK2-average conserves 1/2 v^T M_V v + 1^T M_E e for any force (Sec. 2.2.1), here with piecewise
    rho0 and gamma and the viscosity active behind the waves."""
    wl = W.triple_point((14, 4))
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, 0.3, record=False)
    E = np.array(tr.energy)
    assert len(tr.dt) > 10
    assert np.abs(E - E[0]).max() <= 1e-13 * E[0]
    assert np.abs(tr.v).max() > 0.1  # the shock has started to move


def _tg_noav(n=4):
    mesh = oracle_problem(W.tg2d(n)).mesh
    return F.build_operator(Problem("taylor_green", mesh, 5 / 3, False, 0.5))


def test_rk4_is_fourth_order_in_time():
    op = _tg_noav()
    T = 0.2
    sols = {}
    for k in (8, 16, 32, 128):
        tr = F.run_fom(op, T, fixed_dt=T / (5 * k), record=False, scheme="rk4")
        sols[k] = np.concatenate([tr.x, tr.v, tr.e])
    e1, e2, e4 = (np.linalg.norm(sols[k] - sols[128]) for k in (8, 16, 32))
    # error ratios per halving approach 2^4 (14.97 and 15.9 here; 11.3 at 10 steps, pre-asymptotic)
    assert 14.5 < e1 / e2 < 17.5 and 14.5 < e2 / e4 < 17.5, (e1, e2, e4)


def test_rk4_is_not_the_rk2avg_step_and_one_step_matches_the_butcher_tableau():
    """One RK4 step by hand from the right-hand side: y + dt/6 (k1 + 2 k2 + 2 k3 + k4)."""
    op = _tg_noav()
    y = initial_state(op.prob)
    dt = 0.01

    def f(x, v, e):
        st = F.stress(op, x, v, e)
        return np.concatenate([v, -op.solve_v(F.force_one(op, st)), op.solve_e(F.force_tv(op, st, v))])

    NV = op.mesh.NV
    Y = np.concatenate(y)

    def split(Z):
        return Z[:NV], Z[NV:2 * NV], Z[2 * NV:]

    k1 = f(*split(Y))
    k2 = f(*split(Y + dt / 2 * k1))
    k3 = f(*split(Y + dt / 2 * k2))
    k4 = f(*split(Y + dt * k3))
    expect = Y + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    r = F.rk4_step(op, *y, dt)
    got = np.concatenate([r.x, r.v, r.e])
    assert np.abs(got - expect).max() <= 1e-14 * np.abs(expect).max()
    r2 = F.rk2avg_step(op, *y, dt)
    assert np.abs(np.concatenate([r2.x, r2.v, r2.e]) - expect).max() > 1e-9


@pytest.fixture(scope="module")
def tg_rk4():
    wl = W.tg2d(6)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, 0.05, fixed_dt=2.5e-3, scheme="rk4")
    return wl, op, tr, initial_state(op.prob)


def test_rk4_rom_reproduces_the_rk4_fom_with_full_bases_and_sampling(tg_rk4):
    wl, op, tr, y0 = tg_rk4
    mats = snapshot_matrices([tr], [y0], [0.05])[0]
    ranks = []
    for S in mats:
        s = np.linalg.svd(S, compute_uv=False)
        ranks.append(int(np.sum(s > 1e-11 * s[0])))
    rom = R.build_rom(op, [tr], [y0], [0.05], n_fixed=ranks, lam=(1e9, 1e9))
    run = R.run_rom(op, rom, y0, 0.05, dt_replay=tr.dt, scheme="rk4")
    err = R.relative_errors((tr.x, tr.v, tr.e), R.final_lift(rom, run))
    assert max(err) < 1e-10, err
    # the same bases under RK2-average do not retrace the RK4 trajectory
    run2 = R.run_rom(op, rom, y0, 0.05, dt_replay=tr.dt)
    assert max(R.relative_errors((tr.x, tr.v, tr.e), R.final_lift(rom, run2))) > 1e-8


def test_rk4_rom_is_fourth_order_in_time():
    """Viscosity off (its max(0, .) switches are not smooth in the state), 6 modes per field."""
    op = _tg_noav(6)
    tr = F.run_fom(op, 0.1, fixed_dt=2.5e-3, scheme="rk4")
    y0 = initial_state(op.prob)
    rom = R.build_rom(op, [tr], [y0], [0.1], n_fixed=(6, 6, 6))
    sols = {}
    for k in (4, 8, 16, 64):
        run = R.run_rom(op, rom, y0, 0.1, fixed_dt=0.1 / (4 * k), scheme="rk4")
        sols[k] = np.concatenate(run.yhat)
    e1, e2, e4 = (np.linalg.norm(sols[k] - sols[64]) for k in (4, 8, 16))
    assert 14.0 < e1 / e2 < 18.0 and 14.0 < e2 / e4 < 18.0, (e1, e2, e4)
