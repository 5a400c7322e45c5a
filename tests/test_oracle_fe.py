"""Pins of the oracle's finite-element layer against closed forms (CPU)."""
import json
import os

import numpy as np
import pytest

from oracle.fe import Q1_NODES_1D, Q2_NODES_1D, Mesh, gauss_legendre_01, lagrange_1d, ref_tables

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_lagrange_is_nodal():
    for nodes in (Q2_NODES_1D, Q1_NODES_1D):
        L, _ = lagrange_1d(nodes, nodes)
        np.testing.assert_allclose(L, np.eye(len(nodes)), atol=1e-15)


def test_lagrange_derivative_matches_closed_form():
    xi = np.linspace(0, 1, 7)
    _, dL = lagrange_1d(Q2_NODES_1D, xi)
    # N0 = 2(x-1/2)(x-1), N1 = -4x(x-1), N2 = 2x(x-1/2)
    np.testing.assert_allclose(dL[:, 0], 4 * xi - 3, atol=1e-14)
    np.testing.assert_allclose(dL[:, 1], -8 * xi + 4, atol=1e-14)
    np.testing.assert_allclose(dL[:, 2], 4 * xi - 1, atol=1e-14)


def test_gauss_legendre_exact_to_degree_7():
    x, w = gauss_legendre_01(4)
    for p in range(8):
        assert abs(np.sum(w * x**p) - 1.0 / (p + 1)) < 1e-15
    assert abs(np.sum(w * x**8) - 1.0 / 9) > 1e-6  # and not beyond


@pytest.mark.parametrize("dim", [2, 3])
def test_partition_of_unity(dim):
    R = ref_tables(dim)
    np.testing.assert_allclose(R.B.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(R.dB.sum(axis=1), 0.0, atol=1e-13)
    np.testing.assert_allclose(R.Bt.sum(axis=1), 1.0, atol=1e-14)
    assert abs(R.w.sum() - 1.0) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_reference_gradient_reproduces_linear_map(dim):
    """sum_a X_a dN_a/dxi = identity when X_a are the reference node positions."""
    R = ref_tables(dim)
    loc = np.array([[((a // 3**c) % 3) * 0.5 for c in range(dim)] for a in range(3**dim)])
    J = np.einsum("ac,qai->qci", loc, R.dB)
    np.testing.assert_allclose(J, np.broadcast_to(np.eye(dim), J.shape), atol=1e-14)
    # and interpolates the quadrature point itself
    np.testing.assert_allclose(R.B @ loc, R.xi, atol=1e-15)


def test_dof_counts_match_table_fom():
    """N_V = d (2n+1)^d and N_E = 2^d n^d reproduce the paper's Table tab:fom sizes."""
    with open(os.path.join(GOLDEN, "fom_sizes.json")) as f:
        rows = json.load(f)["rows"]
    for r in rows:
        mesh = Mesh(len(r["nel"]), tuple(r["nel"]), (0.0,) * len(r["nel"]), (1.0,) * len(r["nel"]))
        if r["order"] == 2:
            assert mesh.NV == r["NV"] and mesh.NE == r["NE"], r
        else:
            # Gresho is Q3-Q2 on 32^2 in the paper; Q2-Q1 on 48^2 has the same N_V and N_E.
            assert mesh.NV == r["NV"] and mesh.NE == r["NE"], r


@pytest.mark.parametrize("dim,nel", [(2, (3, 2)), (3, (2, 3, 2))])
def test_connectivity_geometry(dim, nel):
    mesh = Mesh(dim, nel, (0.0,) * dim, (1.0,) * dim)
    X = mesh.node_coords()
    en = mesh.elem_nodes()
    E = mesh.elem_coords()
    h = mesh.h
    for K in range(mesh.n_elem):
        for a in range(3**dim):
            want = [(E[K, c] + 0.5 * ((a // 3**c) % 3)) * h[c] for c in range(dim)]
            np.testing.assert_allclose(X[en[K, a]], want, atol=1e-15)
    # each node appears in 1..2^d elements, corners of the box in exactly one
    counts = np.bincount(en.ravel(), minlength=mesh.n_nodes)
    assert counts.min() == 1 and counts.max() == 2**dim


def test_constrained_dofs_are_wall_normals():
    mesh = Mesh(2, (2, 2), (0.0, 0.0), (1.0, 1.0))
    X = mesh.node_coords()
    m = mesh.constrained_dofs().reshape(2, -1)
    assert np.array_equal(m[0], np.isclose(X[:, 0], 0) | np.isclose(X[:, 0], 1))
    assert np.array_equal(m[1], np.isclose(X[:, 1], 0) | np.isclose(X[:, 1], 1))
