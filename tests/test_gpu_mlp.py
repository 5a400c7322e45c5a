"""MLP surrogate on the GPU against the oracle (MI355X).

Network weights, inputs and normalisation are seeded host data given to
both sides; nothing the GPU computes is fed back to the oracle.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fom as F
from oracle import mlp as M
from oracle import rom as R
from oracle.problems import initial_state
from tests.oracle_adapter import oracle_problem
from tests.test_gpu_rom import _t, gpu_instance, rel

pytestmark = pytest.mark.gpu


def make_net(sizes, seed, scale=1.0, mu_out=None, s_out=None, mu_in=None, s_in=None):
    g = W.rng(seed)
    Ws, _ = M.glorot_init(sizes, g)
    bs = [g.normal(0.0, 0.05, n) for n in sizes[1:]]
    return M.MLP([scale * w for w in Ws], bs,
                 g.normal(0, 1, sizes[0]) if mu_in is None else mu_in,
                 g.uniform(0.5, 2, sizes[0]) if s_in is None else s_in,
                 g.normal(0, 1, sizes[-1]) if mu_out is None else mu_out,
                 g.uniform(0.5, 2, sizes[-1]) if s_out is None else s_out)


def gpu_net(net, max_batch):
    from paper_2104_11404_amd import lib
    m = lib.Mlp(net.sizes, max_batch)
    m.set_params([_t(w) for w in net.W], [_t(b) for b in net.b], _t(net.mu_in), _t(net.s_in), _t(net.mu_out),
                 _t(net.s_out))
    return m


def nrel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_single_layer_matches_oracle_ragged_tiles(gpu_lib):
    print("[case] mlp single layer 61 -> 440, batch 200", flush=True)
    net = make_net([61, 440], 11)
    X = W.rng(12).normal(0, 1, (200, 61))
    m = gpu_net(net, 256)
    Y = m.forward(_t(X)).cpu().numpy()
    assert nrel(Y, M.predict(net, X)) < 1e-6
    # gradients: one layer, so the only bfloat16 roundings are of z_0 and of the output gradient
    # (an FP32 output gradient may round to the other neighbour on a handful of the 88000 entries)
    T = W.rng(13).normal(0, 1, (200, 440))
    gW, gb, loss = m.gradients(_t(X), _t(T))
    oW, ob = M.backward(net, X, T)
    assert nrel(gW[0].cpu().numpy(), oW[0]) < 1e-4
    assert nrel(gb[0].cpu().numpy(), ob[0]) < 1e-5
    assert abs(float(loss) - M.loss(net, X, T)) <= 1e-5 * M.loss(net, X, T)


def test_deep_forward_layer_by_layer_and_end_to_end(gpu_lib):
    sizes = [61, 256, 256, 256, 440]
    print(f"[case] mlp forward {sizes}", flush=True)
    net = make_net(sizes, 21)
    X = W.rng(22).normal(0, 1, (300, 61))
    m = gpu_net(net, 512)
    Y, tr = m.forward(_t(X), trace=True)
    tr = [t.cpu().numpy().astype(np.float64) for t in tr]
    # each layer from the GPU's own input to it
    np.testing.assert_allclose(tr[0], (X - net.mu_in) / net.s_in, rtol=1e-6, atol=1e-6)
    for l in range(len(net.W)):
        z = M.bf16(tr[l]) @ M.bf16(net.W[l]) + net.b[l]
        ref = np.tanh(z) if l < len(net.W) - 1 else z
        assert nrel(tr[l + 1], ref) < 1e-5, l
    # end to end against the oracle's own forward pass
    assert nrel(Y.cpu().numpy(), M.predict(net, X)) < 1e-2


def test_gradients_and_adam_match_oracle(gpu_lib):
    sizes = [13, 64, 48, 20]
    print(f"[case] mlp gradients {sizes}", flush=True)
    net = make_net(sizes, 31)
    g = W.rng(32)
    X = g.normal(0, 1, (150, 13))
    T = g.normal(0, 1, (150, 20))
    m = gpu_net(net, 256)
    gW, gb, loss = m.gradients(_t(X), _t(T))
    oW, ob = M.backward(net, X, T)
    for l in range(3):
        assert nrel(gW[l].cpu().numpy(), oW[l]) < 2e-2, l
        assert nrel(gb[l].cpu().numpy(), ob[l]) < 2e-2, l
    # three Adam steps: the parameter changes agree with the oracle's
    W0 = [w.copy() for w in net.W]
    opt = M.Adam(lr=1e-3)
    for _ in range(3):
        m.train_step(_t(X), _t(T), 1e-3)
        oW, ob = M.backward(net, X, T)
        opt.step(net.W + net.b, oW + ob)
    Wg, bg = m.get_params()
    for l in range(3):
        assert nrel(Wg[l].cpu().numpy() - W0[l], net.W[l] - W0[l]) < 5e-2, l


def test_backward_layer_by_layer_from_the_gpus_own_activations_and_deltas(gpu_lib):
    """Each product of the backward pass from the GPU's own bfloat16-rounded inputs to it: the output
    delta from the GPU's normalised output, D_l = (r(D_{l+1}) r(W_l)^T) (1 - z_l^2), grad W_l =
    r(z_l)^T r(D_{l+1}) and grad b_l = column sums of D_{l+1}, at the FP32 accumulation bound."""
    sizes = [61, 256, 256, 256, 440]
    print(f"[case] mlp backward per layer {sizes}", flush=True)
    net = make_net(sizes, 51)
    g = W.rng(52)
    B = 300
    X = g.normal(0, 1, (B, 61))
    T = g.normal(0, 1, (B, 440)) * net.s_out + net.mu_out
    m = gpu_net(net, 512)
    _, zs = m.forward(_t(X), trace=True)
    gW, gb, _ = m.gradients(_t(X), _t(T))
    D = [d.cpu().numpy().astype(np.float64) for d in m.last_deltas(B)]
    z = [t.cpu().numpy().astype(np.float64) for t in zs]
    L = len(net.W)
    tt = (T - net.mu_out) / net.s_out
    assert nrel(D[L - 1], 2.0 * (z[L] - tt) / (B * sizes[-1])) < 1e-6
    for l in range(L - 1, -1, -1):
        assert nrel(gW[l].cpu().numpy(), M.bf16(z[l]).T @ M.bf16(D[l])) < 1e-5, l
        assert nrel(gb[l].cpu().numpy(), D[l].sum(axis=0)) < 1e-5, l
        if l > 0:
            ref = (M.bf16(D[l]) @ M.bf16(net.W[l]).T) * (1.0 - z[l] ** 2)
            assert nrel(D[l - 1], ref) < 1e-5, l


def test_training_fits_a_teacher_network(gpu_lib):
    from paper_2104_11404_amd import lib
    print("[case] mlp training on a teacher", flush=True)
    teacher = make_net([9, 32, 7], 41, scale=1.5)
    g = W.rng(42)
    X = g.normal(0, 1, (1024, 9))
    T = M.predict(teacher, X, r=M.identity)
    mu_in, s_in = M.normalisation(X)
    mu_out, s_out = M.normalisation(T)
    student = make_net([9, 64, 64, 7], 43, mu_in=mu_in, s_in=s_in, mu_out=mu_out, s_out=s_out)
    m = gpu_net(student, 1024)
    Xt, Tt = _t(X), _t(T)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    m.train_step(Xt, Tt, 3e-3, loss)
    first = float(loss)
    for _ in range(600):
        m.train_step(Xt, Tt, 3e-3, loss)
    last = float(loss)
    print("loss", first, "->", last, flush=True)
    assert last < 0.02 * first


@pytest.fixture(scope="module")
def tg_surrogate():
    wl = W.tg2d(8)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=wl.fixed_dt)
    y0 = initial_state(op.prob)
    rom = R.build_rom(op, [tr], [y0], [wl.t_final], n_fixed=(6, 6, 6), lam=(2, 2))
    X, T = M.training_set(op, rom, 0, [tr], [[0] * len(tr.snaps)])
    return wl, op, tr, y0, rom, X, T


def test_targets_match_oracle(gpu_lib, tg_surrogate):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0, rom, X, T = tg_surrogate
    print("[case] surrogate targets tg2d", flush=True)
    P = lib.Problem.from_workload(wl)
    G = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    idx = np.arange(0, len(X), 7)
    Tg = lib.rom_surrogate_targets(G, 0, 0, _t(X[idx, :-1])).cpu().numpy()
    for r, i in enumerate(idx):
        assert nrel(Tg[r], T[i]) < 1e-10, i


def _surrogate_net(rom, X, T, seed, scale):
    din, dout = M.layout(rom.windows[0])
    mu_in, s_in = M.normalisation(X)
    mu_out, s_out = M.normalisation(T)
    return make_net([din, 64, 64, dout], seed, scale=scale, mu_in=mu_in, s_in=s_in, mu_out=mu_out,
                    s_out=0.05 * s_out)


def test_surrogate_rom_matches_oracle(gpu_lib, tg_surrogate):
    """Fixed steps: same audits and surrogate steps, reduced state within the bfloat16 bound."""
    from paper_2104_11404_amd import lib
    wl, op, tr, y0, rom, X, T = tg_surrogate
    print("[case] surrogate rom tg2d fixed dt", flush=True)
    net = _surrogate_net(rom, X, T, 51, 0.3)
    run = M.run_surrogate(op, rom, {0: net}, y0, wl.t_final, audit_every=10, tol=10.0, fixed_dt=wl.fixed_dt)
    assert run.surrogate_steps == 90 and run.audits == 10 and not run.fallback_windows
    P = lib.Problem.from_workload(wl)
    G = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    m = gpu_net(net, 16)
    G.attach_surrogate(0, 0, m, audit_every=10, tol=10.0)
    G.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]), wl.fixed_dt)
    G.step(flags=lib.LH_SURROGATE | lib.LH_FIXED_DT)
    st = G.states()[0]
    assert st.status == 0 and st.n_steps == len(run.dt)
    assert st.n_audits == run.audits and st.n_surrogate_steps == run.surrogate_steps and st.n_fallbacks == 0
    for a, b in zip(G.coords(0), run.yhat):
        assert rel(a, b) < 1e-3


def test_failed_audit_falls_back_bitwise(gpu_lib, tg_surrogate):
    from paper_2104_11404_amd import lib
    wl, op, tr, y0, rom, X, T = tg_surrogate
    print("[case] surrogate fallback tg2d", flush=True)
    net = _surrogate_net(rom, X, T, 52, 0.3)
    P = lib.Problem.from_workload(wl)
    m = gpu_net(net, 16)
    G = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    G.attach_surrogate(0, 0, m, audit_every=4, tol=-1.0)
    G.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]))
    G.step(flags=lib.LH_SURROGATE)
    st = G.states()[0]
    assert st.n_fallbacks == 1 and st.n_audits == 1 and st.n_surrogate_steps == 0
    G2 = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    G2.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]))
    G2.step()
    s2 = G2.states()[0]
    assert st.n_steps == s2.n_steps and st.t == s2.t
    for a, b in zip(G.coords(0), G2.coords(0)):
        np.testing.assert_array_equal(a, b)


def test_nonfinite_surrogate_step_falls_back_bitwise(gpu_lib, tg_surrogate):
    """A network that is exactly 0 at the zero initial coordinates (the audit passes) and overflows the
    first surrogate step: the non-finite state is caught, the step is redone with DEIM and the rest of the
    window stays on DEIM, as in the oracle; the run is bitwise the plain ROM's."""
    from paper_2104_11404_amd import lib
    from tests.test_oracle_mlp import blowup_net
    wl, op, tr, y0, rom, X, T = tg_surrogate
    print("[case] surrogate non-finite fallback tg2d", flush=True)
    din, dout = M.layout(rom.windows[0])
    net = blowup_net([din, 8, dout])
    with np.errstate(over="ignore", invalid="ignore"):
        run = M.run_surrogate(op, rom, {0: net}, y0, wl.t_final, audit_every=5, tol=1.0)
    assert run.audits == 1 and run.fallback_windows == [0] and run.surrogate_steps == 0
    P = lib.Problem.from_workload(wl)
    G = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    m = gpu_net(net, 16)
    G.attach_surrogate(0, 0, m, audit_every=5, tol=1.0)
    G.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]))
    G.step(flags=lib.LH_SURROGATE)
    st = G.states()[0]
    assert st.status == 0 and st.done == 1
    assert st.n_fallbacks == 1 and st.n_audits == 1 and st.n_surrogate_steps == 0
    G2 = lib.Rom(P, [gpu_instance(rom, wl.t_final)])
    G2.init_state(_t(y0[0]), _t(y0[1]), _t(y0[2]))
    G2.step()
    s2 = G2.states()[0]
    assert st.n_steps == s2.n_steps and st.t == s2.t
    for a, b in zip(G.coords(0), G2.coords(0)):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(G.coords(0), R.run_rom(op, rom, y0, wl.t_final).yhat):
        assert rel(a, b) < 1e-9


def test_trained_network_gains_over_untrained_and_over_deim_work(gpu_lib):
    """Parametric 2D Taylor-Green (16 x 16, A in [0.8, 1.2], 8 instances): the network trained on
    the GPU against the same network untrained, both run without fallback.  The trained one tracks
    the FOM better, and both take a tenth of the DEIM chain's sampled force evaluations."""
    from paper_2104_11404_amd import lib, pipeline
    wl = W.replace(W.tg2d_param(n=16, t_final=0.1, n_inst=8), n_fixed=(10, 10, 10))
    print("[case] trained surrogate gain tg2d 16x16", flush=True)
    trajs = [pipeline.fom_trajectory(lib.Problem.from_workload(wl, amp=A), wl.t_final, fixed_dt=wl.fixed_dt)
             for A in W.TG_TRAIN_AMPS]
    nominal = trajs[1]["y0"]
    P = lib.Problem.from_workload(wl, amp=1.0)
    inst = pipeline.build_offline(P, trajs, [wl.t_final], nominal, n_fixed=wl.n_fixed, lam=wl.lam,
                                  t_final=wl.t_final, snapshot_offsets=nominal)
    y0s, finals = [], []
    for prm in wl.params:
        Pi = lib.Problem.from_workload(wl, amp=prm["amp"])
        x, v, e = Pi.initial_state()
        y0s.append((x.clone(), v.clone(), e.clone()))
        Pi.fom_run(x, v, e, wl.t_final, fixed_dt=wl.fixed_dt, record=False)
        finals.append((x, v, e))
    y0 = [torch.cat([y[f] for y in y0s]) for f in range(3)]
    rom = lib.Rom(P, [inst] * len(wl.params))
    ntr = [pipeline.fom_trajectory(lib.Problem.from_workload(wl, amp=float(A)), wl.t_final, fixed_dt=wl.fixed_dt)
           for A in np.linspace(0.8, 1.2, 9)]
    X = pipeline.surrogate_inputs(rom, 0, 0, ntr)
    untrained, _, _ = pipeline.train_surrogate(rom, 0, 0, X, steps=1, lr=1e-12)
    trained, T, hist = pipeline.train_surrogate(rom, 0, 0, X, steps=1500, lr=2e-3, lr_final=1e-4)
    print("loss", hist[0], "->", hist[-1], flush=True)
    assert hist[-1] < 1e-2 * hist[0]

    def run(net):
        for i in range(len(wl.params)):
            rom.attach_surrogate(i, 0, net, audit_every=10, tol=1e30)
        rom.init_state(*y0, wl.fixed_dt)
        rom.step(flags=lib.LH_FIXED_DT | (lib.LH_SURROGATE if net is not None else 0))
        sts = rom.states()
        assert all(st.status == 0 and st.done == 1 for st in sts)
        err = np.array([[float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(rom.lift(i), finals[i])]
                        for i in range(len(wl.params))]).max(axis=0)
        return err, sum(st.n_force_evals for st in sts)

    e_deim, ev_deim = run(None)
    e_tr, ev_tr = run(trained)
    e_un, ev_un = run(untrained)
    print("max errors (x, v, e): deim", e_deim, "trained", e_tr, "untrained", e_un, flush=True)
    print("sampled force evaluations: deim", ev_deim, "surrogate", ev_tr, flush=True)
    # what training buys over the same network before training (which, with its output
    # normalisation fitted, predicts the mean force): measured 2.9x (v) and 1.4x (e)
    assert e_tr[1] < 0.5 * e_un[1] and e_tr[2] < e_un[2]
    assert ev_tr <= 0.15 * ev_deim


@pytest.mark.parametrize("sizes,batch", [([7, 16, 16, 16, 16, 16, 16, 16, 5], 1), ([3, 9, 2], 1), ([5, 33, 4], 65)],
                         ids=["8-layers-batch-1", "one-hidden-batch-1", "ragged-batch-65"])
def test_network_limits_layer_by_layer(gpu_lib, sizes, batch):
    """The most layers the library takes (8), a batch of one sample and ragged tiles: every layer
    from the GPU's own input to it, and the gradients of a one-sample batch."""
    from paper_2104_11404_amd import lib
    print(f"[case] mlp limits {sizes} batch {batch}", flush=True)
    assert len(sizes) - 1 <= lib.LH_MLP_MAX_LAYERS
    net = make_net(sizes, 31, scale=0.5)
    X = W.rng(32).normal(0, 1, (batch, sizes[0]))
    m = gpu_net(net, max(batch, 2))
    Y, tr = m.forward(_t(X), trace=True)
    tr = [t.cpu().numpy().astype(np.float64) for t in tr]
    for l in range(len(net.W)):
        z = M.bf16(tr[l]) @ M.bf16(net.W[l]) + net.b[l]
        ref = np.tanh(z) if l < len(net.W) - 1 else z
        assert nrel(tr[l + 1], ref) < 1e-5, l
    T = W.rng(33).normal(0, 1, (batch, sizes[-1]))
    gW, gb, loss = m.gradients(_t(X), _t(T))
    oW, ob = M.backward(net, X, T)
    assert nrel(gW[-1].cpu().numpy(), oW[-1]) < 2e-2
    assert nrel(gb[-1].cpu().numpy(), ob[-1]) < 2e-2
