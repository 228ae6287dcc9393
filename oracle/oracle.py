"""Python driver for the plain FP64 CPU oracle in ``oracle.c``.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.
It imports nothing from the HIP package; every function takes plain numpy
arrays (element type code, coordinates, cells, ...).

Element type codes: 1 = Q1 quad, 2 = P1 triangle, 3 = Q1 hexahedron,
4 = P2 (10-node) tetrahedron.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int
_D = ctypes.c_double


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no fast-math;
    OpenMP for the multi-threaded baseline variants only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_element_ke0.restype = _D
        L.oracle_element_ke0.argtypes = [_I32, _P, _D, _I32, _P]
        L.oracle_node_pairs.restype = _I64
        L.oracle_node_pairs.argtypes = [_I32, _I64, _I64, _P, _P]
        L.oracle_pattern_from_pairs.argtypes = [_I32, _I64, _I64, _P, _P, _P]
        L.oracle_assemble.argtypes = [_I32, _I64, _P, _I64, _P, _P, _D, _D, _D, _D, _I32, _P, _P, _P, _P]
        L.oracle_element_energy.argtypes = [_I32, _I64, _P, _I64, _P, _D, _I32, _P, _P]
        L.oracle_sensitivity.argtypes = [_I32, _I64, _P, _I64, _P, _P, _D, _D, _D, _D, _I32, _P, _P]
        L.oracle_compliance.argtypes = [_I32, _I64, _P, _I64, _P, _P, _D, _D, _D, _D, _I32, _P, _P, _P]
        L.oracle_assemble_backward.argtypes = [_I32, _I64, _P, _I64, _P, _P, _D, _D, _D, _D, _I32,
                                               _P, _P, _P, _P]
        L.oracle_spmv.argtypes = [_I64, _P, _P, _P, _P, _P]
        L.oracle_solve_banded.argtypes = [_I64, _P, _P, _P, _P, _I64, _P, _P]
        L.oracle_ref_basis.argtypes = [_I32, _P, _P, _P]
        L.oracle_quadrature.argtypes = [_I32, _P, _P, _P]
        L.oracle_D.argtypes = [_I32, _I32, _D, _D, _P]
        L.oracle_hex27_node.argtypes = [_I32, _P]
        L.oracle_assemble_mt.argtypes = L.oracle_assemble.argtypes
        L.oracle_element_energy_mt.argtypes = L.oracle_element_energy.argtypes
        L.oracle_sensitivity_mt.argtypes = L.oracle_sensitivity.argtypes
        L.oracle_compliance_mt.argtypes = L.oracle_compliance.argtypes
        L.oracle_threads.argtypes = []
        for name in ("oracle_pattern_from_pairs", "oracle_assemble", "oracle_element_energy",
                     "oracle_sensitivity", "oracle_compliance", "oracle_assemble_backward",
                     "oracle_spmv", "oracle_solve_banded", "oracle_ref_basis", "oracle_quadrature",
                     "oracle_D", "oracle_hex27_node", "oracle_assemble_mt", "oracle_element_energy_mt",
                     "oracle_sensitivity_mt", "oracle_compliance_mt", "oracle_threads"):
            getattr(L, name).restype = _I32
        _lib = L
    return _lib


DIM = {1: 2, 2: 2, 3: 3, 4: 3, 5: 3}
NEN = {1: 4, 2: 3, 3: 8, 4: 10, 5: 27}


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


# ----------------------------------------------------------- element level

def element_ke0(elem: int, xe, nu: float = 0.3, plane_strain: int = 0) -> np.ndarray:
    """K_e^0 (unit Young's modulus) of one element with node coordinates xe [nen, dim]."""
    xe = _c(xe, np.float64)
    ldof = DIM[elem] * NEN[elem]
    Ke = np.zeros((ldof, ldof))
    lib().oracle_element_ke0(elem, _ptr(xe), nu, plane_strain, _ptr(Ke))
    return Ke


def D_matrix(dim: int, E: float = 1.0, nu: float = 0.3, plane_strain: int = 0) -> np.ndarray:
    n = 3 if dim == 2 else 6
    D = np.zeros((n, n))
    _check(lib().oracle_D(dim, plane_strain, E, nu, _ptr(D)), "D")
    return D


def ref_basis(elem: int, xi):
    xi = _c(xi, np.float64)
    phi = np.zeros(NEN[elem])
    dphi = np.zeros((NEN[elem], DIM[elem]))
    _check(lib().oracle_ref_basis(elem, _ptr(xi), _ptr(phi), _ptr(dphi)), "ref_basis")
    return phi, dphi


def hex27_node(i: int):
    """Lattice indices (a, b, c) in {0, 1, 2}^3 of the Q2 hexahedron's node i
    (position (a, b, c) / 2 on the reference cube)."""
    abc = np.zeros(3, np.int32)
    _check(lib().oracle_hex27_node(i, _ptr(abc)), "hex27_node")
    return tuple(int(v) for v in abc)


def quadrature(elem: int):
    pts = np.zeros((27, 3))
    wts = np.zeros(27)
    nq = ctypes.c_int(0)
    _check(lib().oracle_quadrature(elem, ctypes.byref(nq), _ptr(pts), _ptr(wts)), "quadrature")
    d = DIM[elem]
    flat = pts.ravel()[: d * nq.value].reshape(nq.value, d)
    return flat.copy(), wts[: nq.value].copy()


# ---------------------------------------------------------------- pattern

def pattern(elem: int, n_nodes: int, cells):
    """CSR pattern (row_ptr int64 [ndof+1], col_idx int32 [nnz]) of the mesh."""
    cells = _c(cells, np.int32)
    nc = cells.shape[0]
    nen = NEN[elem]
    keys = np.empty(max(nc * nen * nen, 1), dtype=np.int64)
    npairs = lib().oracle_node_pairs(elem, n_nodes, nc, _ptr(cells), _ptr(keys))
    if npairs < 0:
        raise RuntimeError("oracle pattern failed")
    d = DIM[elem]
    row_ptr = np.zeros(d * n_nodes + 1, dtype=np.int64)
    col_idx = np.empty(max(npairs * d * d, 1), dtype=np.int32)
    _check(lib().oracle_pattern_from_pairs(d, n_nodes, npairs, _ptr(keys), _ptr(row_ptr), _ptr(col_idx)),
           "pattern")
    return row_ptr, col_idx[: npairs * d * d].copy()


# ------------------------------------------------------------- global ops

def assemble(elem, coords, cells, rho, row_ptr, col_idx, E0=1.0, Emin=1e-9, p=3.0, nu=0.3,
             plane_strain=0, mask=None, mt=False):
    coords, cells, rho = _c(coords, np.float64), _c(cells, np.int32), _c(rho, np.float64)
    row_ptr, col_idx = _c(row_ptr, np.int64), _c(col_idx, np.int32)
    mask = None if mask is None else _c(mask, np.uint8)
    K = np.zeros(col_idx.shape[0])
    fn = lib().oracle_assemble_mt if mt else lib().oracle_assemble
    _check(fn(elem, coords.shape[0], _ptr(coords), cells.shape[0], _ptr(cells), _ptr(rho), E0, Emin, p, nu,
              plane_strain, _ptr(mask), _ptr(row_ptr), _ptr(col_idx), _ptr(K)), "assemble")
    return K


def element_energy(elem, coords, cells, u, nu=0.3, plane_strain=0, mt=False):
    coords, cells, u = _c(coords, np.float64), _c(cells, np.int32), _c(u, np.float64)
    s = np.zeros(cells.shape[0])
    fn = lib().oracle_element_energy_mt if mt else lib().oracle_element_energy
    _check(fn(elem, coords.shape[0], _ptr(coords), cells.shape[0], _ptr(cells), nu, plane_strain, _ptr(u),
              _ptr(s)), "element_energy")
    return s


def sensitivity(elem, coords, cells, rho, u, E0=1.0, Emin=1e-9, p=3.0, nu=0.3, plane_strain=0, mt=False):
    coords, cells = _c(coords, np.float64), _c(cells, np.int32)
    rho, u = _c(rho, np.float64), _c(u, np.float64)
    dc = np.zeros(cells.shape[0])
    fn = lib().oracle_sensitivity_mt if mt else lib().oracle_sensitivity
    _check(fn(elem, coords.shape[0], _ptr(coords), cells.shape[0], _ptr(cells), _ptr(rho), E0, Emin, p, nu,
              plane_strain, _ptr(u), _ptr(dc)), "sensitivity")
    return dc


def compliance(elem, coords, cells, rho, u, f=None, E0=1.0, Emin=1e-9, p=3.0, nu=0.3, plane_strain=0,
               mt=False):
    coords, cells = _c(coords, np.float64), _c(cells, np.int32)
    rho, u = _c(rho, np.float64), _c(u, np.float64)
    f = None if f is None else _c(f, np.float64)
    c = np.zeros(2)
    fn = lib().oracle_compliance_mt if mt else lib().oracle_compliance
    _check(fn(elem, coords.shape[0], _ptr(coords), cells.shape[0], _ptr(cells), _ptr(rho), E0, Emin, p, nu,
              plane_strain, _ptr(u), _ptr(f), _ptr(c)), "compliance")
    return c


def assemble_backward(elem, coords, cells, rho, row_ptr, col_idx, Kbar, E0=1.0, Emin=1e-9, p=3.0,
                      nu=0.3, plane_strain=0):
    coords, cells, rho = _c(coords, np.float64), _c(cells, np.int32), _c(rho, np.float64)
    row_ptr, col_idx, Kbar = _c(row_ptr, np.int64), _c(col_idx, np.int32), _c(Kbar, np.float64)
    drho = np.zeros(cells.shape[0])
    _check(lib().oracle_assemble_backward(elem, coords.shape[0], _ptr(coords), cells.shape[0],
                                          _ptr(cells), _ptr(rho), E0, Emin, p, nu, plane_strain,
                                          _ptr(row_ptr), _ptr(col_idx), _ptr(Kbar), _ptr(drho)),
           "assemble_backward")
    return drho


def threads() -> int:
    """Threads the multi-threaded variants (mt=True) use: OpenMP's maximum."""
    return int(lib().oracle_threads())


def spmv(row_ptr, col_idx, K, x):
    row_ptr, col_idx = _c(row_ptr, np.int64), _c(col_idx, np.int32)
    K, x = _c(K, np.float64), _c(x, np.float64)
    n = row_ptr.shape[0] - 1
    y = np.zeros(n)
    _check(lib().oracle_spmv(n, _ptr(row_ptr), _ptr(col_idx), _ptr(K), _ptr(x), _ptr(y)), "spmv")
    return y


def solve(row_ptr, col_idx, K, f):
    """Banded Cholesky solve of the SPD system K u = f (Dirichlet rows already applied)."""
    row_ptr, col_idx = _c(row_ptr, np.int64), _c(col_idx, np.int32)
    K, f = _c(K, np.float64), _c(f, np.float64)
    n = row_ptr.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    bw = int(np.max(np.abs(rows - col_idx))) if col_idx.size else 0
    band = np.zeros(n * (bw + 1))
    u = np.zeros(n)
    _check(lib().oracle_solve_banded(n, _ptr(row_ptr), _ptr(col_idx), _ptr(K), _ptr(f), bw, _ptr(band),
                                     _ptr(u)), "solve")
    return u
