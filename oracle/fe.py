"""Finite-element spaces of the semi-discretisation (oracle, test infrastructure).

The paper discretises the Lagrangian Euler equations with a continuous
kinematic space (positions and velocities) and a discontinuous thermodynamic
space (specific internal energy), the Q_k - Q_{k-1} pair of Dobrev et al.
(Sec. 2.1, "Spatial discretization"; Table tab:fom gives k = 2 or 3).  This
oracle implements k = 2 on uniform Cartesian meshes of [lo, hi]^d, d = 2, 3:

* kinematic space: continuous Q2 Lagrange, 1D nodes {0, 1/2, 1} on the
  reference interval [0, 1];
* thermodynamic space: discontinuous Q1 Lagrange at the two Gauss-Legendre
  points 1/2 -+ sqrt(3)/6 (the paper does not name the Q1 basis; any choice
  leaves sum_j phi_j = 1, which is all the method uses of it);
* quadrature: tensor Gauss-Legendre with 4 points per direction for both the
  force and the mass integrals (the paper mentions quadrature points in
  eq. adaptive-timestep but not the rule).

Numbering (shared by every array in the oracle):

* local Q2 node a = i + 3 j (+ 9 k), x fastest; local Q1 dof j likewise in
  base 2; quadrature point q = qx + 4 qy (+ 16 qz);
* global node (gx, gy[, gz]) with gx = 2 ex + i, id = gx + Nx (gy + Ny gz),
  Nx = 2 nx + 1;
* kinematic vector: component-major, entry c * Nnodes + node;
* thermodynamic vector: element-major, entry K * 2^d + j with
  K = ex + nx (ey + ny ez).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

Q2_NODES_1D = np.array([0.0, 0.5, 1.0])
Q1_NODES_1D = np.array([0.5 - np.sqrt(3.0) / 6.0, 0.5 + np.sqrt(3.0) / 6.0])
NQ1D = 4
ORDER = 2  # k of the Q_k - Q_{k-1} pair


def lagrange_1d(nodes: np.ndarray, xi: np.ndarray):
    """Values and first derivatives of the Lagrange polynomials on ``nodes``.

    Returns (L, dL) with L[p, i] = l_i(xi_p), dL[p, i] = l_i'(xi_p), written
    straight from the product definition l_i = prod_{m != i} (x - x_m)/(x_i - x_m).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    n = len(nodes)
    L = np.ones((len(xi), n))
    dL = np.zeros((len(xi), n))
    for i in range(n):
        others = [m for m in range(n) if m != i]
        denom = np.prod([nodes[i] - nodes[m] for m in others])
        for m in others:
            L[:, i] *= xi - nodes[m]
        L[:, i] /= denom
        # product rule
        for skip in others:
            term = np.ones(len(xi))
            for m in others:
                if m != skip:
                    term *= xi - nodes[m]
            dL[:, i] += term / denom
    return L, dL


def gauss_legendre_01(n: int):
    """n-point Gauss-Legendre rule mapped from [-1, 1] to [0, 1]."""
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


@dataclass(frozen=True)
class RefTables:
    """Tensor-product tables at the quadrature points of the reference cell."""

    dim: int
    B: np.ndarray  # (nq, nk)      Q2 shape values N_a(q)
    dB: np.ndarray  # (nq, nk, d)  reference gradients dN_a/dxi_i at q
    Bt: np.ndarray  # (nq, nt)     Q1 shape values phi_j(q)
    w: np.ndarray  # (nq,)         quadrature weights on [0,1]^d
    xi: np.ndarray  # (nq, d)      quadrature points on [0,1]^d


def ref_tables(dim: int) -> RefTables:
    xq, wq = gauss_legendre_01(NQ1D)
    Lk, dLk = lagrange_1d(Q2_NODES_1D, xq)  # (4, 3)
    Lt, _ = lagrange_1d(Q1_NODES_1D, xq)  # (4, 2)
    qidx = list(itertools.product(range(NQ1D), repeat=dim))  # tuples, first index slowest
    qidx = [tuple(reversed(t)) for t in qidx]  # (qx, qy[, qz]) with qx fastest
    kidx = [tuple(reversed(t)) for t in itertools.product(range(3), repeat=dim)]
    tidx = [tuple(reversed(t)) for t in itertools.product(range(2), repeat=dim)]
    nq, nk, nt = len(qidx), len(kidx), len(tidx)
    B = np.ones((nq, nk))
    dB = np.ones((nq, nk, dim))
    Bt = np.ones((nq, nt))
    w = np.ones(nq)
    xi = np.zeros((nq, dim))
    for q, qq in enumerate(qidx):
        for c in range(dim):
            w[q] *= wq[qq[c]]
            xi[q, c] = xq[qq[c]]
        for a, aa in enumerate(kidx):
            for c in range(dim):
                B[q, a] *= Lk[qq[c], aa[c]]
            for i in range(dim):
                for c in range(dim):
                    dB[q, a, i] *= dLk[qq[c], aa[c]] if c == i else Lk[qq[c], aa[c]]
        for j, jj in enumerate(tidx):
            for c in range(dim):
                Bt[q, j] *= Lt[qq[c], jj[c]]
    return RefTables(dim, B, dB, Bt, w, xi)


@dataclass(frozen=True)
class Mesh:
    """Uniform Cartesian mesh of [lo, hi]^d with Q2 nodes and Q1 dofs."""

    dim: int
    nel: tuple
    lo: tuple
    hi: tuple

    @property
    def h(self) -> np.ndarray:
        return (np.array(self.hi, float) - np.array(self.lo, float)) / np.array(self.nel, float)

    @property
    def nodes_per_dir(self) -> tuple:
        return tuple(2 * n + 1 for n in self.nel)

    @property
    def n_nodes(self) -> int:
        return int(np.prod(self.nodes_per_dir))

    @property
    def n_elem(self) -> int:
        return int(np.prod(self.nel))

    @property
    def NV(self) -> int:
        """Kinematic dof count N_V = d (2n+1)^d."""
        return self.dim * self.n_nodes

    @property
    def NE(self) -> int:
        """Thermodynamic dof count N_E = 2^d n^d."""
        return (2 ** self.dim) * self.n_elem

    def node_coords(self) -> np.ndarray:
        """(n_nodes, d) reference positions of the Q2 nodes."""
        axes = [np.linspace(self.lo[c], self.hi[c], self.nodes_per_dir[c]) for c in range(self.dim)]
        grids = np.meshgrid(*axes, indexing="ij")  # grids[c][gx, gy, ...]
        # flatten with x fastest: transpose so that the last axis is x
        return np.stack([g.transpose(tuple(reversed(range(self.dim)))).ravel() for g in grids], axis=1)

    def elem_coords(self):
        """(n_elem, d) integer element coordinates (ex, ey[, ez]), x fastest."""
        rng = [range(n) for n in self.nel]
        return np.array([tuple(reversed(t)) for t in itertools.product(*reversed(rng))], dtype=np.int64)

    def elem_nodes(self) -> np.ndarray:
        """(n_elem, 3^d) global node ids of each element, local a = i + 3j (+9k)."""
        E = self.elem_coords()
        Nd = self.nodes_per_dir
        loc = [tuple(reversed(t)) for t in itertools.product(range(3), repeat=self.dim)]
        out = np.zeros((self.n_elem, len(loc)), dtype=np.int64)
        for a, aa in enumerate(loc):
            g = [2 * E[:, c] + aa[c] for c in range(self.dim)]
            idx = g[0].copy()
            stride = 1
            for c in range(1, self.dim):
                stride *= Nd[c - 1]
                idx += stride * g[c]
            out[:, a] = idx
        return out

    def elem_thermo(self) -> np.ndarray:
        """(n_elem, 2^d) thermodynamic dof ids of each element."""
        nt = 2 ** self.dim
        return np.arange(self.n_elem)[:, None] * nt + np.arange(nt)[None, :]

    def constrained_dofs(self) -> np.ndarray:
        """Boolean mask over the N_V kinematic dofs fixed by v.n = 0 on the walls.

        Dof (c, node) is constrained when the node lies on a face of the box
        whose normal is e_c (all benchmark problems use wall conditions on
        every face, Sec. 6.1).
        """
        X = self.node_coords()
        mask = np.zeros(self.NV, dtype=bool)
        for c in range(self.dim):
            on = np.isclose(X[:, c], self.lo[c]) | np.isclose(X[:, c], self.hi[c])
            mask[c * self.n_nodes:(c + 1) * self.n_nodes] = on
        return mask

    def node_elements(self):
        """List over nodes of the sorted element ids that contain the node."""
        en = self.elem_nodes()
        out = [[] for _ in range(self.n_nodes)]
        for K in range(self.n_elem):
            for a in en[K]:
                out[a].append(K)
        return [sorted(set(v)) for v in out]
