"""Pins of the MLP-surrogate oracle (oracle/mlp.py) against things other than itself."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fom as F
from oracle import mlp as M
from oracle import rom as R
from oracle.problems import initial_state
from tests.oracle_adapter import oracle_problem


def small_net(sizes, seed=3, scale=1.0):
    g = np.random.default_rng(seed)
    Ws, bs = M.glorot_init(sizes, g)
    bs = [g.normal(0, 0.1, b.shape) for b in bs]
    return M.MLP([scale * w for w in Ws], bs, g.normal(0, 1, sizes[0]), g.uniform(0.5, 2, sizes[0]),
                 g.normal(0, 1, sizes[-1]), g.uniform(0.5, 2, sizes[-1]))


def test_bf16_rounding_matches_torch_and_ties_to_even():
    g = np.random.default_rng(0)
    x = np.concatenate([g.normal(0, 1, 2000), g.normal(0, 1e6, 500), g.normal(0, 1e-6, 500),
                        [0.0, -0.0, 1.0, np.inf, -np.inf, 3.0e38, 1e-40]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)
    # exact ties: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 and goes to the even one (1)
    assert M.bf16(1.0 + 2.0 ** -8) == 1.0
    assert M.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert np.isnan(M.bf16(np.nan))


def test_backward_matches_central_differences():
    net = small_net([5, 7, 6, 4])
    g = np.random.default_rng(1)
    X = g.normal(0, 1, (9, 5))
    T = g.normal(0, 1, (9, 4))
    gW, gb = M.backward(net, X, T, r=M.identity)
    h = 1e-6
    for l in range(3):
        for arr, grad in ((net.W[l], gW[l]), (net.b[l], gb[l])):
            num = np.zeros_like(arr)
            for idx in np.ndindex(arr.shape):
                old = arr[idx]
                arr[idx] = old + h
                lp = M.loss(net, X, T, r=M.identity)
                arr[idx] = old - h
                lm = M.loss(net, X, T, r=M.identity)
                arr[idx] = old
                num[idx] = (lp - lm) / (2 * h)
            assert np.linalg.norm(num - grad) <= 1e-7 * np.linalg.norm(grad)


def test_bf16_backward_rounds_only_the_product_operands():
    """With every operand already a bfloat16 value the rounded and exact paths agree."""
    net = small_net([4, 8, 3])
    net.W = [M.bf16(w) for w in net.W]
    net.mu_in, net.s_in = np.zeros(4), np.ones(4)
    X = M.bf16(np.random.default_rng(2).normal(0, 1, (6, 4)))
    a_r = M.forward(net, X, r=M.bf16)
    a_i = M.forward(net, X, r=M.identity)
    np.testing.assert_array_equal(a_r[1], a_i[1])  # first layer: operands exact in bfloat16


def test_zero_weights_give_the_bias_and_normalisation_is_standard():
    net = small_net([3, 5, 2])
    net.W = [np.zeros_like(w) for w in net.W]
    X = np.random.default_rng(4).normal(0, 3, (7, 3))
    np.testing.assert_allclose(M.predict(net, X), np.tile(net.mu_out + net.s_out * net.b[-1], (7, 1)))
    mu, s = M.normalisation(X)
    Z = (X - mu) / s
    np.testing.assert_allclose(Z.mean(axis=0), 0, atol=1e-15)
    np.testing.assert_allclose(Z.std(axis=0), 1, rtol=1e-14)
    _, s0 = M.normalisation(np.ones((4, 2)))
    assert np.all(s0 == 1.0)


def test_adam_first_steps_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    g1 = np.array([0.3, -1e-3, 0.0])
    opt = M.Adam(lr=0.01)
    q = p.copy()
    opt.step([q], [g1])
    # bias-corrected first step: m^ = g, v^ = g^2
    np.testing.assert_allclose(q, p - 0.01 * g1 / (np.abs(g1) + 1e-8), rtol=1e-15, atol=1e-18)
    g2 = np.array([-0.1, 2e-3, 1.0])
    q2 = q.copy()
    opt.step([q2], [g2])
    m = 0.9 * 0.1 * g1 + 0.1 * g2
    v = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    np.testing.assert_allclose(q2, q - 0.01 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8),
                               rtol=1e-14)


@pytest.fixture(scope="module")
def tg_rom():
    wl = W.tg2d(6)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, 0.03, fixed_dt=1e-3)
    y0 = initial_state(op.prob)
    rom = R.build_rom(op, [tr], [y0], [0.03], n_fixed=(5, 5, 5), lam=(2, 2))
    return op, tr, y0, rom


def test_targets_are_the_deim_chain_and_linear_in_the_contraction_velocity(tg_rom):
    op, tr, y0, rom = tg_rom
    win = rom.windows[0]
    g = np.random.default_rng(5)
    yh = tuple(0.1 * g.normal(0, 1, n) for n in win.dims)
    f1, ff, H = M.split_output(win, M.deim_targets(op, win, yh))
    # F^1 as the ROM step uses it: v_{1/2} = v^ - dt/2 F^1
    dt = 1e-4
    _, half, _ = R.rom_step(op, win, *yh, dt)
    np.testing.assert_allclose((yh[1] - half[1]) / (0.5 * dt), f1, rtol=1e-9, atol=1e-12)
    # F^tv for an arbitrary contraction velocity, evaluated the ROM's way (lift, then contract)
    NV, NE = op.mesh.NV, op.mesh.NE
    st = F.stress(op, R.lift_rows(win, 0, yh[0], win.rows_k, NV), R.lift_rows(win, 1, yh[1], win.rows_k, NV),
                  R.lift_rows(win, 2, yh[2], win.rows_t, NE), elems=win.elems)
    for vc in [yh[1]] + [g.normal(0, 1, win.dims[1]) for _ in range(3)]:
        direct = win.A2 @ F.force_tv(op, st, R.lift_rows(win, 1, vc, win.rows_k, NV), elems=win.elems)[win.Z2]
        np.testing.assert_allclose(ff + H @ (vc - yh[1]), direct, rtol=1e-10, atol=1e-12 * np.linalg.norm(direct))


def test_surrogate_step_with_exact_targets_is_the_deim_step(tg_rom, monkeypatch):
    op, tr, y0, rom = tg_rom
    win = rom.windows[0]
    yh = tuple(0.05 * np.random.default_rng(6).normal(0, 1, n) for n in win.dims)

    def exact(net, X, r=None):
        row = X[0]
        nx, nv, ne = win.dims
        return M.deim_targets(op, win, (row[:nx], row[nx:nx + nv], row[nx + nv:nx + nv + ne]))[None, :]

    monkeypatch.setattr(M, "predict", exact)
    dt = 2e-4
    got = M.surrogate_step(win, None, *yh, 0.0, dt)
    ref, _, _ = R.rom_step(op, win, *yh, dt)
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)


def test_failed_audit_falls_back_to_the_plain_rom(tg_rom):
    op, tr, y0, rom = tg_rom
    din, dout = M.layout(rom.windows[0])
    net = small_net([din, 8, dout])
    run = M.run_surrogate(op, rom, {0: net}, y0, 0.03, audit_every=5, tol=-1.0)
    ref = R.run_rom(op, rom, y0, 0.03)
    assert run.fallback_windows == [0] and run.audits == 1 and run.surrogate_steps == 0
    assert run.dt == ref.dt
    for a, b in zip(run.yhat, ref.yhat):
        np.testing.assert_array_equal(a, b)


def blowup_net(sizes, seed=4):
    """A network that outputs exactly 0 at the all-zero input (zero biases, tanh(0) = 0) and, through an
    output scale of 1e300, overflows the first surrogate step elsewhere: an audit at the zero initial
    coordinates (initial-state offsets, t = 0) passes, the next step's state is not finite."""
    g = np.random.default_rng(seed)
    Ws, bs = M.glorot_init(sizes, g)
    return M.MLP(Ws, [np.zeros_like(b) for b in bs], np.zeros(sizes[0]), np.ones(sizes[0]), np.zeros(sizes[-1]),
                 np.full(sizes[-1], 1e300))


def test_nonfinite_surrogate_state_falls_back_and_redoes_the_step(tg_rom):
    op, tr, y0, rom = tg_rom
    din, dout = M.layout(rom.windows[0])
    net = blowup_net([din, 8, dout])
    nv = rom.windows[0].dims[1]
    with np.errstate(over="ignore", invalid="ignore"):
        new = M.surrogate_step(rom.windows[0], net, *(0.01 * np.ones(n) for n in rom.windows[0].dims), 1e-3, 1e-3)
        assert not all(np.all(np.isfinite(c)) for c in new)
        run = M.run_surrogate(op, rom, {0: net}, y0, 0.03, audit_every=5, tol=1.0)
    ref = R.run_rom(op, rom, y0, 0.03)
    assert run.audits == 1 and run.fallback_windows == [0] and run.surrogate_steps == 0, (run.audits, nv)
    assert run.dt == ref.dt
    for a, b in zip(run.yhat, ref.yhat):
        np.testing.assert_array_equal(a, b)


def test_training_set_inputs_are_projected_snapshots(tg_rom):
    op, tr, y0, rom = tg_rom
    win = rom.windows[0]
    X, T = M.training_set(op, rom, 0, [tr], [[0] * len(tr.snaps)])
    din, dout = M.layout(win)
    assert X.shape == (len(tr.snaps), din) and T.shape == (len(tr.snaps), dout)
    np.testing.assert_allclose(X[:, -1], tr.snap_t, rtol=1e-15)
    j = 7
    x, v, e = tr.snaps[j]
    np.testing.assert_allclose(X[j, :win.dims[0]], win.Phi[0].T @ (x - win.os[0]), rtol=1e-12, atol=1e-15)


def test_audit_of_exact_targets_has_no_discrepancy(tg_rom, monkeypatch):
    op, tr, y0, rom = tg_rom
    win = rom.windows[0]
    yh = tuple(0.05 * np.random.default_rng(8).normal(0, 1, n) for n in win.dims)

    def exact(net, X, r=None):
        row = X[0]
        nx, nv, ne = win.dims
        return M.deim_targets(op, win, (row[:nx], row[nx:nx + nv], row[nx + nv:nx + nv + ne]))[None, :]

    monkeypatch.setattr(M, "predict", exact)
    new, tau, disc = M.audit(op, win, None, yh, 0.0, 2e-4)
    ref, _, tau_ref = R.rom_step(op, win, *yh, 2e-4)
    assert disc < 1e-12 and tau == tau_ref
    for a, b in zip(new, ref):
        np.testing.assert_array_equal(a, b)
