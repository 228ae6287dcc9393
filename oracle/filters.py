"""Plain FP64 CPU oracle of the filter step (Sec. 2.4): the filter matrix
H, the sensitivity filter, the density filter with its chain rule and the
Heaviside projection with its chain rule.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.
It imports nothing from the HIP package.

Definitions followed (Sec. 2.4):
* H_ij = max(0, r_min - dist(i, j)), dist = Euclidean distance of the element
  centroids; N_i = { j : H_ij > 0 } (i itself included, H_ii = r_min);
* sensitivity filter  dc~_i = sum_j H_ij rho_j dc_j / (max(gamma, rho_i) sum_j H_ij),
  gamma = 1e-3;
* density filter      rho~_i = sum_j H_ij v_j rho_j / sum_j H_ij v_j, v_j = element volume;
  its chain rule      dpsi/drho_j = sum_i H_ij v_j / (sum_k H_ik v_k) dpsi/drho~_i;
* Heaviside           rho_bar = 1 - exp(-beta rho~) + rho~ exp(-beta),
  its chain rule      dpsi/drho~ = dpsi/drho_bar (beta exp(-beta rho~) + exp(-beta)).

The neighbour sets are found by brute force over all pairs (in row blocks),
which is what the definition says; it is meant for meshes of up to a few
ten thousand elements.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

GAMMA = 1e-3
# corner (vertex) nodes per element type: Q1 quad, P1 triangle, Q1 hex, P2 tet,
# Q2 hex (its corners are nodes 0-7)
N_VERTEX = {1: 4, 2: 3, 3: 8, 4: 4, 5: 8}


def centroids(elem: int, coords, cells) -> np.ndarray:
    """Element centroids: the mean of the vertex nodes, summed in local order
    (c = x_0; c += x_1; ...; c /= n_vertex)."""
    coords = np.asarray(coords, np.float64)
    cells = np.asarray(cells)
    nv = N_VERTEX[elem]
    c = coords[cells[:, 0]].copy()
    for a in range(1, nv):
        c += coords[cells[:, a]]
    return c / nv


def volumes(elem: int, coords, cells) -> np.ndarray:
    """Element measures v_e = int_e 1 dx = sum_q w_q |det J_e(xi_q)| with the
    element's own quadrature rule (exact for the element maps used here)."""
    coords = np.asarray(coords, np.float64)
    cells = np.asarray(cells)
    pts, wts = O.quadrature(elem)
    v = np.zeros(cells.shape[0])
    for xi, w in zip(pts, wts):
        _, dphi = O.ref_basis(elem, xi)           # [nen, dim]
        J = np.einsum("eaj,am->ejm", coords[cells], dphi)   # dx_j / dxi_m
        v += w * np.abs(np.linalg.det(J))
    return v


def filter_matrix(cent, rmin: float, block: int = 2048):
    """CSR of H over the centroids: (row_ptr int64, col int32 ascending, w float64).
    dist_ij = sqrt(sum_a (c_i,a - c_j,a)^2), squares added in axis order."""
    cent = np.asarray(cent, np.float64)
    n, d = cent.shape
    rows, cols, vals = [], [], []
    for i0 in range(0, n, block):
        ci = cent[i0:i0 + block]
        diff = ci[:, None, 0] - cent[None, :, 0]
        s = diff * diff
        for a in range(1, d):
            diff = ci[:, None, a] - cent[None, :, a]
            s = s + diff * diff
        w = rmin - np.sqrt(s)
        ii, jj = np.nonzero(w > 0.0)          # row-major: rows, then ascending j
        rows.append(ii + i0)
        cols.append(jj)
        vals.append(w[ii, jj])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols).astype(np.int32)
    vals = np.concatenate(vals)
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr), cols, vals


def filter_rows(cent, rmin: float, rows):
    """Rows `rows` of H alone (for meshes too large for the whole matrix):
    a list of (columns ascending, weights), by the same brute force."""
    cent = np.asarray(cent, np.float64)
    d = cent.shape[1]
    out = []
    for i in rows:
        diff = cent[i, 0] - cent[:, 0]
        s = diff * diff
        for a in range(1, d):
            diff = cent[i, a] - cent[:, a]
            s = s + diff * diff
        w = rmin - np.sqrt(s)
        j = np.nonzero(w > 0.0)[0]
        out.append((j.astype(np.int32), w[j]))
    return out


def h_product(H, x) -> np.ndarray:
    """y = H x, each row summed in ascending column order."""
    row_ptr, col, w = H
    return O.spmv(row_ptr, col, w, x)


def sensitivity_filter(H, rho, dc, gamma: float = GAMMA) -> np.ndarray:
    rho = np.asarray(rho, np.float64)
    num = h_product(H, rho * np.asarray(dc, np.float64))
    hs = h_product(H, np.ones_like(rho))
    return num / (np.maximum(gamma, rho) * hs)


def density_filter(H, v, rho) -> np.ndarray:
    v = np.asarray(v, np.float64)
    return h_product(H, v * np.asarray(rho, np.float64)) / h_product(H, v)


def density_filter_backward(H, v, g_tilde) -> np.ndarray:
    """dpsi/drho from dpsi/drho~: v_j sum_i H_ij g_i / (sum_k H_ik v_k).
    H is symmetric, so the sum over i is row j of H."""
    v = np.asarray(v, np.float64)
    return v * h_product(H, np.asarray(g_tilde, np.float64) / h_product(H, v))


def heaviside(rho_tilde, beta: float) -> np.ndarray:
    rt = np.asarray(rho_tilde, np.float64)
    return 1.0 - np.exp(-beta * rt) + rt * np.exp(-beta)


def heaviside_grad(rho_tilde, beta: float) -> np.ndarray:
    """d rho_bar / d rho~."""
    rt = np.asarray(rho_tilde, np.float64)
    return beta * np.exp(-beta * rt) + np.exp(-beta)
