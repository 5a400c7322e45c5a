"""GPU parity of rom_build_basis (POD) and rom_sample_deim (MI355X)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import deim as D
from oracle import fom as F
from oracle.pod import energy_dimension, pod_basis
from oracle.problems import initial_state
from oracle.windows import snapshot_matrices
from tests.oracle_adapter import oracle_problem

pytestmark = pytest.mark.gpu


def _rows(a):
    """N x m column-major matrix as a contiguous (m, N) device tensor."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)).cuda()


def _align(A, B):
    """Flip columns of A to best match B (signs are a convention)."""
    s = np.sign(np.sum(A * B, axis=0))
    s[s == 0] = 1
    return A * s


def _decaying(N, m, seed, rate=0.6, rank=None):
    rng = np.random.default_rng(seed)
    r = rank or m
    U = np.linalg.qr(rng.normal(size=(N, r)))[0]
    V = np.linalg.qr(rng.normal(size=(m, r)))[0]
    s = rate ** np.arange(r)
    return (U * s) @ V.T, s


@pytest.fixture(scope="module")
def tg_snapshots():
    wl = W.tg2d(8)
    op = F.build_operator(oracle_problem(wl))
    tr = F.run_fom(op, wl.t_final, fixed_dt=wl.fixed_dt)
    return op, snapshot_matrices([tr], [initial_state(op.prob)], [wl.t_final])[0]


@pytest.mark.parametrize("N,m,seed", [(700, 60, 0), (1031, 33, 1), (257, 257, 2), (300, 1, 3), (9000, 150, 4),
                                      (4099, 97, 5), (64, 5, 6), (500, 8, 7), (500, 9, 8)])
def test_pod_matches_oracle_random(gpu_lib, N, m, seed):
    from paper_2104_11404_amd import lib
    print(f"[case] pod random N={N} m={m}", flush=True)
    S, _ = _decaying(N, m, seed, rate=0.7)
    nfix = min(10, m)
    Phi_g, sig_g, n = lib.rom_build_basis(_rows(S), n_fixed=nfix)
    Phi_o, sig_o, _ = pod_basis(S, n_fixed=nfix)
    assert n == nfix
    sig_g = sig_g.cpu().numpy()
    assert np.linalg.norm(sig_g - sig_o) <= 1e-10 * np.linalg.norm(sig_o)
    Pg = Phi_g.cpu().numpy().T
    for k in range(n):
        assert np.linalg.norm(Pg[:, k] - Phi_o[:, k]) < 1e-10, k
    np.testing.assert_allclose(Pg.T @ Pg, np.eye(n), atol=1e-13)


def test_pod_block_and_pair_jacobi_agree(gpu_lib, monkeypatch):
    """The block Jacobi sweep (2 x 8 columns in LDS) and the one-pair rounds reach the same singular
    values and leading vectors."""
    from paper_2104_11404_amd import lib
    S, _ = _decaying(6000, 211, 9, rate=0.8)
    print("[case] pod block against pair Jacobi N=6000 m=211", flush=True)
    Pb, sb, _ = lib.rom_build_basis(_rows(S), n_fixed=12)
    monkeypatch.setenv("LAGROM_POD_JACOBI", "pairs")
    Pp, sp, _ = lib.rom_build_basis(_rows(S), n_fixed=12)
    monkeypatch.delenv("LAGROM_POD_JACOBI")
    sb, sp = sb.cpu().numpy(), sp.cpu().numpy()
    assert np.max(np.abs(sb - sp)) <= 1e-13 * sp[0]
    Pb, Pp = Pb.cpu().numpy(), Pp.cpu().numpy()
    for k in range(12):
        assert min(np.linalg.norm(Pb[k] - Pp[k]), np.linalg.norm(Pb[k] + Pp[k])) < 1e-10, k


def test_pod_energy_criterion_and_eckart_young_on_snapshots(gpu_lib, tg_snapshots):
    from paper_2104_11404_amd import lib
    op, mats = tg_snapshots
    for f, S in enumerate(mats):
        print(f"[case] pod tg2d snapshots field {f}", flush=True)
        Phi_g, sig_g, n = lib.rom_build_basis(_rows(S), energy_frac=0.9999, n_max=64)
        Phi_o, sig_o, n_o = pod_basis(S, energy_frac=0.9999, n_max=64)
        assert n == n_o
        sig_g = sig_g.cpu().numpy()
        assert np.linalg.norm(sig_g - sig_o) <= 1e-10 * np.linalg.norm(sig_o)
        Pg = _align(Phi_g.cpu().numpy().T, Phi_o)
        gaps = np.abs(np.diff(sig_o[: n + 1])) / sig_o[0]
        for k in range(n):
            if min(gaps[max(k - 1, 0)], gaps[k]) > 1e-6:
                assert np.linalg.norm(Pg[:, k] - Phi_o[:, k]) < 1e-9, (f, k)
        resid = np.linalg.norm(S - Pg @ (Pg.T @ S)) ** 2
        assert abs(resid - np.sum(sig_o[n:] ** 2)) <= 1e-10 * np.sum(sig_o**2)


def test_pod_rank_deficient(gpu_lib):
    from paper_2104_11404_amd import lib
    S, s = _decaying(400, 30, 5, rate=0.5, rank=6)
    Phi_g, sig_g, n = lib.rom_build_basis(_rows(S), energy_frac=1.0 - 1e-12)
    sig_g = sig_g.cpu().numpy()
    assert np.all(sig_g[6:] < 1e-13 * sig_g[0])
    np.testing.assert_allclose(sig_g[:6], s, rtol=1e-12)


@pytest.mark.parametrize("N,n,ns,seed", [(500, 8, 8, 0), (500, 8, 13, 1), (731, 12, 30, 2), (300, 5, 300, 3)])
def test_deim_matches_oracle_random(gpu_lib, N, n, ns, seed):
    from paper_2104_11404_amd import lib
    print(f"[case] deim random N={N} n={n} ns={ns}", flush=True)
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.normal(size=(N, n)))[0]
    idx, pinv = lib.rom_sample_deim(_rows(U), ns)
    Zo = D.greedy_deim(U, ns)
    np.testing.assert_array_equal(idx.cpu().numpy(), Zo)
    Ao = D.deim_pinv(U, Zo)
    Ag = pinv.cpu().numpy().T  # rows of the (ns, n) tensor are columns of the n x ns matrix
    assert np.linalg.norm(Ag - Ao) <= 1e-10 * np.linalg.norm(Ao)


def test_deim_sns_basis_with_zero_rows_and_ties(gpu_lib, tg_snapshots):
    """SNS basis of the symmetric TG problem: constrained rows are zero, mirrored rows tie."""
    from paper_2104_11404_amd import lib
    op, mats = tg_snapshots
    for f, lam in ((1, 2), (2, 2), (1, 5)):
        Phi, _, _ = pod_basis(mats[f], n_fixed=6)
        U = op.Mv_eff @ Phi if f == 1 else op.Me @ Phi
        ns = lam * 6
        print(f"[case] deim sns field {f} ns={ns}", flush=True)
        idx, pinv = lib.rom_sample_deim(_rows(U), ns)
        Zo = D.greedy_deim(U, ns)
        np.testing.assert_array_equal(idx.cpu().numpy(), Zo)
        Ao = D.deim_pinv(U, Zo)
        assert np.linalg.norm(pinv.cpu().numpy().T - Ao) <= 1e-10 * np.linalg.norm(Ao)


def test_deim_rank_deficiency_reported(gpu_lib):
    from paper_2104_11404_amd import lib
    rng = np.random.default_rng(4)
    U = rng.normal(size=(200, 4))
    U[:, 3] = 0.0
    with pytest.raises(lib.LagromError) as ei:
        lib.rom_sample_deim(_rows(U), 8)
    assert ei.value.code == -7


@pytest.mark.parametrize("N,n,ns,seed", [(500, 8, 8, 0), (500, 8, 19, 1), (731, 12, 30, 2), (300, 5, 300, 3),
                                         (4099, 20, 123, 4)])
def test_qdeim_matches_oracle_random(gpu_lib, N, n, ns, seed):
    """Q-DEIM indices bit-exact with the oracle: one round (n_s = n), ragged rounds, all rows."""
    from paper_2104_11404_amd import lib
    print(f"[case] qdeim random N={N} n={n} ns={ns}", flush=True)
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.normal(size=(N, n)))[0]
    idx, pinv = lib.rom_sample_qdeim(_rows(U), ns)
    Zo = D.qdeim(U, ns)
    np.testing.assert_array_equal(idx.cpu().numpy(), Zo)
    Ao = D.deim_pinv(U, Zo)
    assert np.linalg.norm(pinv.cpu().numpy().T - Ao) <= 1e-10 * np.linalg.norm(Ao)


def test_qdeim_sns_basis_with_zero_rows_and_ties(gpu_lib, tg_snapshots):
    from paper_2104_11404_amd import lib
    op, mats = tg_snapshots
    for f, lam in ((1, 1), (2, 2), (1, 5)):
        Phi, _, _ = pod_basis(mats[f], n_fixed=6)
        U = op.Mv_eff @ Phi if f == 1 else op.Me @ Phi
        ns = lam * 6
        print(f"[case] qdeim sns field {f} ns={ns}", flush=True)
        idx, pinv = lib.rom_sample_qdeim(_rows(U), ns)
        Zo = D.qdeim(U, ns)
        np.testing.assert_array_equal(idx.cpu().numpy(), Zo)
        Ao = D.deim_pinv(U, Zo)
        assert np.linalg.norm(pinv.cpu().numpy().T - Ao) <= 1e-10 * np.linalg.norm(Ao)
