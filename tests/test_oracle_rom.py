"""Pins of the oracle's POD, DEIM, windows and ROM (CPU)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import deim as D
from oracle import fom as F
from oracle import rom as R
from oracle.pod import canonical_signs, energy_dimension, pod_basis
from oracle.problems import initial_state
from oracle.windows import first_reaching, snapshot_matrices, window_columns, window_start_states, windows_by_samples
from tests.oracle_adapter import oracle_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- POD

def test_pod_eckart_young_and_orthonormality():
    rng = np.random.default_rng(1)
    S = rng.normal(size=(300, 40)) @ np.diag(0.7 ** np.arange(40)) @ rng.normal(size=(40, 40))
    for n in (1, 5, 17):
        Phi, sigma, k = pod_basis(S, n_fixed=n)
        assert k == n
        np.testing.assert_allclose(Phi.T @ Phi, np.eye(n), atol=1e-13)
        resid = np.linalg.norm(S - Phi @ (Phi.T @ S)) ** 2
        assert abs(resid - np.sum(sigma[n:] ** 2)) <= 1e-12 * np.sum(sigma**2)


def test_energy_criterion_uses_sigma_sum():
    sigma = np.array([4.0, 3.0, 2.0, 1.0])  # total 10
    assert energy_dimension(sigma, 0.7) == 2
    assert energy_dimension(sigma, 0.71) == 3
    assert energy_dimension(sigma, 0.9) == 3
    assert energy_dimension(sigma, 0.91) == 4
    # with sigma^2 the answer for 0.9 would be 2 (16+9 of 30 = 0.83 -> 3 ... differs at 0.8)
    assert energy_dimension(sigma, 0.8) == 3


def test_canonical_signs():
    P = np.array([[0.1, -0.5], [-0.9, 0.5], [0.2, 0.1]])
    C = canonical_signs(P)
    np.testing.assert_array_equal(C[:, 0], -P[:, 0])
    np.testing.assert_array_equal(C[:, 1], -P[:, 1])  # tie |-0.5| = |0.5|: first row decides


# ---------------------------------------------------------------- DEIM

def _lu_pivot_order(U):
    lu, piv = sla.lu_factor(U)
    perm = np.arange(U.shape[0])
    for i, p in enumerate(piv):
        perm[i], perm[p] = perm[p], perm[i]
    return perm[: U.shape[1]]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_classic_deim_equals_row_pivoted_lu(seed):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.normal(size=(60, 8)))[0]
    Z = D.greedy_deim(U, 8)
    np.testing.assert_array_equal(Z, _lu_pivot_order(U))


def test_interpolation_exactness_and_projector():
    rng = np.random.default_rng(5)
    N, n = 80, 6
    U = np.linalg.qr(rng.normal(size=(N, n)))[0]
    Z = D.greedy_deim(U, n)
    A = D.deim_pinv(U, Z)
    P = U @ A @ np.eye(N)[Z, :]
    f = rng.normal(size=N)
    np.testing.assert_allclose((P @ f)[Z], f[Z], atol=1e-12)  # n_s = n: interpolation
    np.testing.assert_allclose(P @ P, P, atol=1e-11)
    g = U @ rng.normal(size=n)
    np.testing.assert_allclose(P @ g, g, atol=1e-12)


@pytest.mark.parametrize("ns", [6, 9, 13, 30])
def test_oversampled_projector_and_error_bound(ns):
    rng = np.random.default_rng(7)
    N, n = 90, 6
    U = rng.normal(size=(N, n))
    Z = D.greedy_deim(U, ns)
    assert len(Z) == ns and len(set(Z.tolist())) == ns
    A = D.deim_pinv(U, Z)
    P = U @ A @ np.eye(N)[Z, :]
    np.testing.assert_allclose(P @ P, P, atol=1e-10)
    g = U @ rng.normal(size=n)
    np.testing.assert_allclose(P @ g, g, atol=1e-11)
    Q = np.linalg.qr(U)[0]
    kappa = np.linalg.norm(np.linalg.pinv(Q[Z, :]), 2)
    for _ in range(5):
        f = rng.normal(size=N)
        lhs = np.linalg.norm(f - P @ f)
        rhs = kappa * np.linalg.norm(f - Q @ (Q.T @ f))
        assert lhs <= rhs * (1 + 1e-10)


def test_oversampling_least_squares_matches_normal_equations():
    rng = np.random.default_rng(9)
    U = rng.normal(size=(50, 4))
    Z = D.greedy_deim(U, 11)
    A = D.deim_pinv(U, Z)
    ZU = U[Z]
    np.testing.assert_allclose(A, np.linalg.solve(ZU.T @ ZU, ZU.T), atol=1e-12)


def test_rows_per_iteration_and_printed_sample_counts():
    with open(os.path.join(GOLDEN, "sampling_counts.json")) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        ns1 = min(r["NV"], int(r["lam"][0] * r["nv"]))
        ns2 = min(r["NE"], int(r["lam"][1] * r["ne"]))
        assert [ns1, ns2] == r["ns"], r
        assert sum(D.rows_per_iteration(r["nv"], ns1)) == ns1
    assert D.rows_per_iteration(4, 10) == [3, 3, 2, 2]


def test_ties_go_to_smallest_index_and_zero_rows_last():
    U = np.zeros((8, 1))
    U[[2, 5], 0] = 1.0
    U[[4], 0] = 0.5
    Z = D.greedy_deim(U, 4)
    np.testing.assert_array_equal(Z, [2, 5, 4, 0])


def test_rank_deficient_sampling_is_reported():
    U = np.zeros((6, 2))
    U[0, 0] = 1.0
    U[0, 1] = 1.0
    with pytest.raises(D.RankDeficient):
        D.deim_pinv(U, np.array([0, 1]))


# ---------------------------------------------------------------- windows

def test_window_counts_reproduce_table_tw():
    with open(os.path.join(GOLDEN, "window_counts.json")) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        t = list(np.linspace(0.0, 1.0, r["Nt"] + 1))
        T = windows_by_samples([t], r["Nsample"])
        assert len(T) == r["Nw"], r
        assert len(T) == math.ceil(2 * r["Nt"] / r["Nsample"])


def test_windows_by_samples_takes_earliest_parameter():
    ta = list(np.linspace(0, 1, 11))  # 10 steps
    tb = list(np.linspace(0, 1, 21))  # 20 steps
    T = windows_by_samples([ta, tb], 8)  # 4 steps per window
    assert abs(T[0] - tb[4]) < 1e-15  # param b reaches 4 new steps first
    assert T[-1] == 1.0


def test_window_columns_count():
    class Tr:
        t = list(np.linspace(0, 1, 13))
    cols = window_columns(Tr, [0.25, 0.5, 1.0])
    s = [0] + [first_reaching(Tr.t, T) for T in (0.25, 0.5, 1.0)]
    for w, c in enumerate(cols):
        assert len(c) == 2 * (s[w + 1] - s[w]) + (1 if w > 0 else 0)


# ---------------------------------------------------------------- ROM

@pytest.fixture(scope="module")
def tg_fom():
    wl = W.tg2d(8)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=wl.fixed_dt)
    return wl, op, tr, initial_state(op.prob)


def test_rom_reproduces_fom_with_full_bases_and_sampling(tg_fom):
    """n = rank(S), n_s = N: the hyper-reduced ROM retraces the FOM (Sec. 3, SNS)."""
    wl, op, tr, y0 = tg_fom
    mats = snapshot_matrices([tr], [y0], [wl.t_final])[0]
    ranks = []
    for S in mats:
        s = np.linalg.svd(S, compute_uv=False)
        ranks.append(int(np.sum(s > 1e-11 * s[0])))
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=ranks, lam=(1e9, 1e9))
    assert len(rom.windows[0].elems) == op.mesh.n_elem
    run = R.run_rom(op, rom, y0, wl.t_final, dt_replay=tr.dt)
    err = R.relative_errors((tr.x, tr.v, tr.e), R.final_lift(rom, run))
    assert max(err) < 1e-10, err


def test_rom_initial_coordinates_vanish_with_initial_offsets(tg_fom):
    wl, op, tr, y0 = tg_fom
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(6, 6, 6))
    for c in R.initial_coords(rom, y0):
        assert np.all(c == 0.0)


def test_identical_window_bases_switch_is_identity(tg_fom):
    wl, op, tr, y0 = tg_fom
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(6, 6, 6))
    w0 = rom.windows[0]
    w1 = R.WindowROM(**{**w0.__dict__})
    w1.trans = [(w1.Phi[f].T @ w0.Phi[f], w1.Phi[f].T @ (w0.os[f] - w1.os[f])) for f in range(3)]
    rom2 = R.ROM([w0, w1])
    y = tuple(np.arange(1.0, 7.0) * (f + 1) for f in range(3))
    for a, b in zip(R.switch_window(rom2, 1, y), y):
        np.testing.assert_allclose(a, b, atol=1e-14)


def test_plain_rom_is_accurate_on_tg(tg_fom):
    wl, op, tr, y0 = tg_fom
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=wl.n_fixed, lam=wl.lam)
    w = rom.windows[0]
    assert (len(w.Z1), len(w.Z2)) == (12, 12)
    run = R.run_rom(op, rom, y0, wl.t_final, fixed_dt=wl.fixed_dt)
    err = R.relative_errors((tr.x, tr.v, tr.e), R.final_lift(rom, run))
    assert max(err) < 1e-3, err


def test_rom_windows_reproduce_with_full_rank(tg_fom):
    """Two windows by sample count, full rank and full sampling: still the FOM trajectory."""
    wl, op, tr, y0 = tg_fom
    T = windows_by_samples([tr.t], 2 * 50)
    assert len(T) == 2
    mats = snapshot_matrices([tr], [y0], T)
    ranks = []
    for S in mats[0] + mats[1]:
        s = np.linalg.svd(S, compute_uv=False)
        ranks.append(int(np.sum(s > 1e-11 * s[0])))
    # per-window ranks differ; use the largest of each field's pair, capped by its column count
    rk = [max(ranks[f], ranks[3 + f]) for f in range(3)]
    wins = []
    for w in range(2):
        nf = [min(rk[f], mats[w][f].shape[1], int(np.sum(np.linalg.svd(mats[w][f], compute_uv=False) > 1e-11 * np.linalg.svd(mats[w][f], compute_uv=False)[0]))) for f in range(3)]
        wins.append(R.build_window(op, mats[w], y0, T[w], 0.9999, nf, (1e9, 1e9)))
    wins[1].trans = [(wins[1].Phi[f].T @ wins[0].Phi[f], wins[1].Phi[f].T @ (wins[0].os[f] - wins[1].os[f])) for f in range(3)]
    rom = R.ROM(wins)
    run = R.run_rom(op, rom, y0, wl.t_final, dt_replay=tr.dt)
    assert run.w == 1
    err = R.relative_errors((tr.x, tr.v, tr.e), R.final_lift(rom, run))
    assert max(err) < 1e-9, err


def test_rom_second_order_in_time(tg_fom):
    """Fixed bases and samples: the fully discrete ROM converges at second order in dt."""
    wl, op, tr, y0 = tg_fom
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(6, 6, 6))
    T = 0.05
    sols = []
    for k in (2, 4, 8, 32):
        run = R.run_rom(op, rom, y0, T, fixed_dt=T / (5 * k))
        sols.append(np.concatenate(run.yhat))
    e = [np.linalg.norm(s - sols[-1]) for s in sols[:3]]
    assert 3.3 < e[0] / e[1] < 4.8 and 3.3 < e[1] / e[2] < 4.8, e


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_qdeim_equals_lapack_column_pivoted_qr(seed):
    """n_s = n: the pivots of the QR with column pivoting of U^T (LAPACK geqp3 through SciPy)."""
    rng = np.random.default_rng(seed)
    N, n = 70, 9
    U = rng.normal(size=(N, n))
    piv = sla.qr(U.T, pivoting=True, mode="r")[1]
    np.testing.assert_array_equal(D.qdeim(U, n), piv[:n])


def test_qdeim_meets_its_a_priori_bound_and_finds_a_permuted_identity():
    """||(Z^T U)^{-1}||_2 <= sqrt(n (N - n + 1)) sqrt(4^n + 6n - 1) / 3 for orthonormal U (the bound
    of QR with column pivoting that Q-DEIM inherits), and a basis of unit vectors is sampled at its
    unit entries."""
    rng = np.random.default_rng(11)
    for N, n in ((200, 6), (120, 10)):
        U = np.linalg.qr(rng.normal(size=(N, n)))[0]
        Z = D.qdeim(U, n)
        bound = np.sqrt(n * (N - n + 1)) * np.sqrt(4.0 ** n + 6 * n - 1) / 3
        assert np.linalg.norm(np.linalg.inv(U[Z, :]), 2) <= bound
    perm = np.array([17, 3, 40, 8, 29])
    E = np.eye(50)[:, perm]
    assert set(D.qdeim(E, 5).tolist()) == set(perm.tolist())


@pytest.mark.parametrize("ns", [12, 17, 25])
def test_qdeim_rounds_oversample_with_disjoint_well_posed_rows(ns):
    """n_s > n: rounds of pivoted QR restarted from U, each skipping the rows already chosen; every
    full round's rows alone interpolate (U[Z_round, :] invertible) and the projector is exact on
    range(U)."""
    rng = np.random.default_rng(13)
    N, n = 90, 6
    U = rng.normal(size=(N, n))
    Z = D.qdeim(U, ns)
    assert len(Z) == ns and len(set(Z.tolist())) == ns
    np.testing.assert_array_equal(Z[:n], D.qdeim(U, n))
    for r in range(ns // n):
        assert np.linalg.cond(U[Z[r * n:(r + 1) * n], :]) < 1e8
    A = D.deim_pinv(U, Z)
    g = U @ rng.normal(size=n)
    np.testing.assert_allclose(U @ (A @ g[Z]), g, atol=1e-10)
    np.testing.assert_array_equal(D.qdeim(U, N), np.arange(N))


def test_oblique_window_initial_condition():
    """eq. ic2-tw: with M = I it is eq. ic-tw; a lifted state inside the new window's affine space is
    recovered exactly by both; otherwise it gives the smallest M-norm error of the lifted initial
    state, which the orthogonal projection does not."""
    rng = np.random.default_rng(17)
    N, n_old, n_new = 60, 5, 7
    Phi_old = np.linalg.qr(rng.normal(size=(N, n_old)))[0]
    Phi_new = np.linalg.qr(rng.normal(size=(N, n_new)))[0]
    os_old, os_new = rng.normal(size=N), rng.normal(size=N)
    B = rng.normal(size=(N, N))
    M = B @ B.T + N * np.eye(N)  # symmetric positive definite
    T0, c0 = R.window_transition(Phi_new, os_new, Phi_old, os_old)
    T1, c1 = R.window_transition(Phi_new, os_new, Phi_old, os_old, np.eye(N))
    np.testing.assert_allclose(T1, T0, atol=1e-13)
    np.testing.assert_allclose(c1, c0, atol=1e-13)
    # a lifted state in os_new + span(Phi_new): offsets that differ inside the new span, an old window
    # that contains the new one
    a = rng.normal(size=n_new)
    z = rng.normal(size=n_new)
    os_in = os_new + Phi_new @ a
    Phi_in = np.column_stack([Phi_old, Phi_new])
    coef = np.concatenate([np.zeros(n_old), z - a])  # os_in + Phi_in coef = os_new + Phi_new z
    for Mx in (None, M):
        T2, c2 = R.window_transition(Phi_new, os_new, Phi_in, os_in, Mx)
        np.testing.assert_allclose(T2 @ coef + c2, z, atol=1e-10)
    # generic state: the oblique coordinates minimise the M-norm of the error
    yh = rng.normal(size=n_old)
    y = os_old + Phi_old @ yh
    Tm, cm = R.window_transition(Phi_new, os_new, Phi_old, os_old, M)
    Mnorm = lambda e: float(np.sqrt(e @ M @ e))
    best = Mnorm(y - os_new - Phi_new @ (Tm @ yh + cm))
    for _ in range(20):
        d = 1e-3 * rng.normal(size=n_new)
        assert Mnorm(y - os_new - Phi_new @ (Tm @ yh + cm + d)) >= best
    assert Mnorm(y - os_new - Phi_new @ (T0 @ yh + c0)) > best


def test_idw_weights_of_the_interpolated_offsets():
    """eq. interpolate_os with r = 2: hand values for three scalar parameters, a convex combination,
    exact at training parameters, symmetric between two equidistant ones."""
    w = R.idw_weights([0.8, 1.0, 1.2], 0.9)
    np.testing.assert_allclose(w, np.array([100.0, 100.0, 1 / 0.09]) / (200.0 + 1 / 0.09), rtol=1e-14)
    np.testing.assert_array_equal(R.idw_weights([0.8, 1.0, 1.2], 1.2), [0.0, 0.0, 1.0])
    w = R.idw_weights([[0.0, 0.0], [2.0, 0.0]], [1.0, 3.0])
    np.testing.assert_allclose(w, [0.5, 0.5], rtol=1e-15)
    assert abs(R.idw_weights([0.8, 1.0, 1.2], 1.37).sum() - 1.0) < 1e-15
    offs = [[(np.full(3, k + 1.0), np.zeros(3), np.ones(2)) for k in range(3)] for _ in range(2)]
    got = R.interpolated_offsets(offs, [0.8, 1.0, 1.2], 0.9)
    np.testing.assert_allclose(got[1][0], np.full(3, w_dot := float(np.dot(R.idw_weights([0.8, 1.0, 1.2], 0.9),
                                                                          [1.0, 2.0, 3.0]))), rtol=1e-15)
    np.testing.assert_allclose(got[0][2], np.ones(2), rtol=1e-15)


def test_window_start_offsets_are_the_trajectory_states_at_window_starts():
    """The window-start offsets are the step states that close the previous windows, so each window's
    first snapshot column (that state) is the zero deviation; the first window starts at y0."""
    wl = W.tg2d(4)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, 0.02, fixed_dt=1e-3)
    y0 = initial_state(op.prob)
    T = [0.007, 0.014, 0.02]
    starts = window_start_states(tr, y0, T)
    for f in range(3):
        np.testing.assert_array_equal(starts[0][f], y0[f])
    mats = snapshot_matrices([tr], [y0], T, offsets_by_window=[[s] for s in starts])
    for w in (1, 2):
        for f in range(3):
            assert np.abs(mats[w][f][:, 0]).max() == 0.0
    rom = R.build_rom(op, [tr], [y0], T, n_fixed=(3, 3, 3), lam=(2, 2), window_offsets="window_start",
                      online_offsets=starts)
    for w in range(3):
        for f in range(3):
            np.testing.assert_array_equal(rom.windows[w].os[f], starts[w][f])


def test_previous_window_offsets_retrace_the_fom_with_full_bases(tg_fom):
    """eq. previous_os: with window-start training offsets, bases of full rank in every window and
    full sampling, the ROM whose next offset is its own lifted state at each switch retraces the FOM
    through several windows (the lifted state at a switch is the FOM state, which is the training
    offset the next window was built around); the reduced state restarts at zero at every switch."""
    wl, op, tr, y0 = tg_fom
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 3)))
    assert len(T) == 3
    starts = window_start_states(tr, y0, T)
    mats = snapshot_matrices([tr], [y0], T, offsets_by_window=[[s] for s in starts])
    ranks = [max(int(np.sum(np.linalg.svd(S, compute_uv=False) > 1e-11 * np.linalg.norm(S, 2))), 1)
             for S in mats[0]]
    rom = R.build_rom(op, [tr], [y0], T, n_fixed=ranks, lam=(1e9, 1e9), window_offsets="window_start",
                      online_offsets=starts)
    run = R.run_rom(op, rom, y0, wl.t_final, dt_replay=tr.dt, offsets="previous")
    assert run.w == 2
    err = R.relative_errors((tr.x, tr.v, tr.e), R.final_lift(rom, run))
    assert max(err) < 1e-9, err
    # the offsets in use at the end are the ROM's own lifted state at the last switch, i.e. the FOM's
    for f in range(3):
        np.testing.assert_allclose(run.os[f], starts[2][f], rtol=1e-9, atol=1e-12)


def test_mass_orthonormal_basis_is_gram_schmidt_in_the_mass_inner_product():
    """Sec. 3.2 (eq. rmass, reduced mass I): Phi^T M Phi = I, the same subspace, and column k equals
    the M-normalised part of phi_k M-orthogonal to phi_1..phi_{k-1} (modified Gram-Schmidt in the M
    inner product, written out here); M = I leaves an orthonormal basis unchanged."""
    rng = np.random.default_rng(23)
    N, n = 50, 6
    Phi = np.linalg.qr(rng.normal(size=(N, n)))[0]
    B = rng.normal(size=(N, N))
    M = B @ B.T + N * np.eye(N)
    Q = R.mass_orthonormal(Phi, M)
    np.testing.assert_allclose(Q.T @ M @ Q, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(Phi @ (Phi.T @ Q), Q, atol=1e-12)  # inside span(Phi)
    G = Phi.copy()
    for k in range(n):
        for j in range(k):
            G[:, k] -= (G[:, j] @ M @ G[:, k]) * G[:, j]
        G[:, k] /= np.sqrt(G[:, k] @ M @ G[:, k])
    np.testing.assert_allclose(Q, G, atol=1e-11)
    np.testing.assert_allclose(R.mass_orthonormal(Phi, np.eye(N)), Phi, atol=1e-14)


def test_mass_orthonormal_rom_equals_the_euclidean_basis_rom_with_full_sampling(tg_fom):
    """Same subspaces, projections in the mass inner product (eq. ic2-tw for the window changes): with
    every element sampled the reduced dynamics do not depend on the basis of each subspace, so the
    lifted states of the two ROMs agree through three windows at reduced rank."""
    wl, op, tr, y0 = tg_fom
    T = windows_by_samples([tr.t], 2 * int(np.ceil(len(tr.dt) / 3)))
    kw = dict(n_fixed=(5, 6, 4), lam=(1e9, 1e9), window_ic="oblique")
    rom_e = R.build_rom(op, [tr], [y0], T, **kw)
    rom_m = R.build_rom(op, [tr], [y0], T, basis="mass", **kw)
    for w in rom_m.windows:
        np.testing.assert_allclose(w.Phi[1].T @ op.Mv_eff @ w.Phi[1], np.eye(6), atol=1e-10)
        np.testing.assert_allclose(w.Phi[2].T @ op.Me @ w.Phi[2], np.eye(4), atol=1e-10)
    run_e = R.run_rom(op, rom_e, y0, wl.t_final, dt_replay=tr.dt)
    run_m = R.run_rom(op, rom_m, y0, wl.t_final, dt_replay=tr.dt)
    assert run_m.w == len(T) - 1
    for a, b in zip(R.final_lift(rom_m, run_m), R.final_lift(rom_e, run_e)):
        assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)


def test_mass_basis_initial_coordinates_are_the_mass_projection(tg_fom):
    """With an offset other than the initial state the first coordinates are the M-orthogonal
    projection: the residual y0 - os - Phi yhat is M-orthogonal to the window's basis."""
    wl, op, tr, y0 = tg_fom
    shifted = (y0[0], y0[1] * 0.9, y0[2] * 1.1)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(4, 5, 3), window_ic="oblique", basis="mass",
                      online_offsets=shifted)
    yh = R.initial_coords(rom, y0)
    win = rom.windows[0]
    for f, M in ((1, op.Mv_eff), (2, op.Me)):
        r = y0[f] - win.os[f] - win.Phi[f] @ yh[f]
        assert np.max(np.abs(win.Phi[f].T @ (M @ r))) <= 1e-10 * max(1.0, np.linalg.norm(M @ r))
    with pytest.raises(ValueError):
        R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(4, 5, 3), basis="mass")
