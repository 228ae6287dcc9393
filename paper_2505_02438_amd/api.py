"""Python binding of libsoptx (argument marshalling only).

Torch tensors serve as device buffers and torch streams as HIP streams; every
step of assembly, sensitivity, compliance and backward runs in the library's
HIP kernels.  The names mirror the C ABI in include/soptx.h.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import numpy as np

from . import _lib
from ._lib import BF16_FP32ACC, FP32, FP64, REF_QUADRATURE, REF_SYMBOLIC, check, lib

__all__ = ["Material", "Pattern", "Dirichlet", "FP64", "FP32", "BF16_FP32ACC", "REF_SYMBOLIC", "REF_QUADRATURE",
           "reference_tensor", "validate_mesh", "host_plan"]

_DIM = {1: 2, 2: 2, 3: 3, 4: 3, 5: 3}
_NEN = {1: 4, 2: 3, 3: 8, 4: 10, 5: 27}


@dataclasses.dataclass
class Material:
    """Linear elastic SIMP material (Sec. 2.1, Sec. 3.2.1): E0, Emin, nu, p."""
    E0: float = 1.0
    Emin: float = 1e-9
    nu: float = 0.3
    p: float = 3.0
    plane_strain: int = 0

    def _c(self) -> _lib.Material:
        return _lib.Material(self.E0, self.Emin, self.nu, self.p, self.plane_strain)


def _mesh_struct(elem: int, coords: np.ndarray, cells: np.ndarray):
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    m = _lib.Mesh(elem, _DIM.get(elem, 0), coords.shape[0], coords.ctypes.data, cells.shape[0], cells.ctypes.data)
    return m, (coords, cells)


def reference_tensor(elem: int, method: int = REF_SYMBOLIC) -> np.ndarray:
    """M[i, j, m, n] = int_ref d_m phi_i d_n phi_j (host only)."""
    d, n = _DIM[elem], _NEN[elem]
    M = np.zeros((n, n, d, d))
    check(lib().soptx_reference_tensor(elem, method, M.ctypes.data), "soptx_reference_tensor")
    return M


def validate_mesh(elem: int, coords, cells) -> int:
    """Status code of the library's mesh validation (host only)."""
    m, keep = _mesh_struct(elem, coords, cells)
    return lib().soptx_validate_mesh(ctypes.byref(m))


def host_plan(elem: int, coords, cells, general: bool = False) -> dict:
    """Host-side pattern, geometry and assembly plan as numpy arrays (copies);
    general: the plan of soptx_build_pattern_general, with its contribution
    table (gptr, gent, gnode)."""
    m, keep = _mesh_struct(elem, coords, cells)
    L = lib()
    h = ctypes.c_void_p()
    check(L.soptx_debug_host_plan_ex(ctypes.byref(m), 1 if general else 0, ctypes.byref(h)), "soptx_debug_host_plan")
    try:
        out = {}
        dt = {4: np.int32, 2: np.uint16, 1: np.uint8, 8: np.float64}
        for name in ("row_ptr", "col_idx", "geo", "sig_info", "sig_pos_ptr", "sig_contrib", "sig_pairs", "sig_witems", "sig_witem_ptr",
                     "grp_info", "grp_nodes", "grp_elems", "grp_n2l", "grp_rows", "grp_rank_off", "grp_rank", "elem_by_rank", "pos", "nb_tslot",
                     "nb_tdeg",
                     "gptr", "gent", "gnode", "qgeo"):
            ptr, cnt, eb = ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_int32()
            check(L.soptx_debug_host_plan_array(h, name.encode(), ctypes.byref(ptr), ctypes.byref(cnt),
                                                ctypes.byref(eb)), name)
            dtype = np.float64 if name in ("geo", "qgeo") else dt[eb.value]
            if cnt.value == 0:
                out[name] = np.zeros(0, dtype=dtype)
            else:
                buf = (ctypes.c_char * (cnt.value * eb.value)).from_address(ptr.value)
                out[name] = np.frombuffer(buf, dtype=dtype).copy()
        sc = np.zeros(8, dtype=np.int64)
        check(L.soptx_debug_host_plan_scalars(h, sc.ctypes.data), "scalars")
        out.update(dict(zip(["ndof", "nnz", "n_groups", "n_signatures", "emax", "kmax", "dim", "nen"],
                            [int(x) for x in sc])))
        return out
    finally:
        L.soptx_debug_host_plan_free(h)


def _stream_ptr(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _on(stream):
    """Context in which a call allocates its default outputs: the call's own
    stream, so that the allocation (and a fill such as torch.zeros) is
    ordered with the library's kernels on that stream."""
    import contextlib
    import torch
    if stream is None:
        return contextlib.nullcontext()
    if not isinstance(stream, torch.cuda.Stream):
        stream = torch.cuda.ExternalStream(int(stream))
    return torch.cuda.stream(stream)


def _dptr(t, name, dtype=None, numel=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


class Pattern:
    """A mesh's CSR pattern, geometry and assembly plan, resident on the device.

    Built once per mesh (Sec. 3.2.2: invariant components are cached);
    assemble / sensitivity / compliance / backward run per call.
    """

    def __init__(self, elem: int, coords, cells, ref_method: int = REF_SYMBOLIC, general: bool = False,
                 stream=None):
        m, keep = _mesh_struct(elem, coords, cells)
        h = ctypes.c_void_p()
        if general:
            check(lib().soptx_build_pattern_general(ctypes.byref(m), ctypes.byref(h), _stream_ptr(stream)),
                  "soptx_build_pattern_general")
        else:
            check(lib().soptx_build_pattern_ex(ctypes.byref(m), ref_method, ctypes.byref(h), _stream_ptr(stream)),
                  "soptx_build_pattern")
        self.general = general
        self._h = h
        self.elem = elem
        self.dim = _DIM[elem]
        self.nen = _NEN[elem]
        self.n_nodes = int(keep[0].shape[0])
        self.n_cells = int(keep[1].shape[0])
        ndof, nnz = ctypes.c_int64(), ctypes.c_int64()
        check(lib().soptx_pattern_info(h, ctypes.byref(ndof), ctypes.byref(nnz), None, None), "pattern_info")
        self.ndof, self.nnz = ndof.value, nnz.value

    @classmethod
    def from_mesh(cls, mesh, **kw) -> "Pattern":
        return cls(mesh.elem, mesh.coords, mesh.cells, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().soptx_destroy_pattern(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self) -> dict:
        s = _lib.PatternStats()
        check(lib().soptx_pattern_stats_get(self._h, ctypes.byref(s)), "stats")
        return {f: getattr(s, f) for f, _ in s._fields_}

    def pattern(self):
        """(row_ptr, col_idx) copied to host numpy int32 arrays."""
        rp = np.zeros(self.ndof + 1, dtype=np.int32)
        ci = np.zeros(max(self.nnz, 1), dtype=np.int32)
        check(lib().soptx_pattern_copy(self._h, rp.ctypes.data, ci.ctypes.data), "soptx_pattern_copy")
        return rp, ci[: self.nnz]

    # ------------------------------------------------------------- per call
    def _rho_dtype(self, prec):
        import torch
        return torch.float64 if prec == FP64 else torch.float32

    def assemble(self, material: Material, rho, mask=None, out=None, prec: int = FP64, stream=None):
        """K values (FP64, [nnz]) = sum_e E(rho_e) K_e^0 (Eq. cmpd), Dirichlet rows/cols if mask."""
        import torch
        if out is None:
            with _on(stream):
                out = torch.empty(self.nnz, dtype=torch.float64, device=rho.device)
        mc = material._c()
        check(lib().soptx_assemble(self._h, ctypes.byref(mc), _dptr(rho, "rho", self._rho_dtype(prec), self.n_cells),
                                   _dptr(mask, "mask", torch.uint8, self.ndof),
                                   _dptr(out, "out", torch.float64, self.nnz), prec, _stream_ptr(stream)),
              "soptx_assemble")
        return out

    def assemble_general(self, material: Material, rho, mask=None, out=None, stream=None):
        """K = sum_e E(rho_e) K_e^0 with K_e^0 integrated at the quadrature points
        (Q1, affine or not; patterns built with general=True), FP64."""
        import torch
        if out is None:
            with _on(stream):
                out = torch.empty(self.nnz, dtype=torch.float64, device=rho.device)
        mc = material._c()
        check(lib().soptx_assemble_general(self._h, ctypes.byref(mc), _dptr(rho, "rho", torch.float64, self.n_cells),
                                           _dptr(mask, "mask", torch.uint8, self.ndof),
                                           _dptr(out, "K", torch.float64, self.nnz), _stream_ptr(stream)),
              "soptx_assemble_general")
        return out

    def evaluate_general(self, material: Material, rho, u, f=None, dc=None, c=None, stream=None):
        """(dc, c) with the Jacobian at every Gauss point (patterns built with
        general=True), FP64: dc_e = -E'(rho_e) u_e^T K_e^0 u_e, c = [u^T K u, f^T u]."""
        import torch
        if dc is None:
            with _on(stream):
                dc = torch.empty(self.n_cells, dtype=torch.float64, device=rho.device)
        if c is None:
            with _on(stream):
                c = torch.zeros(2, dtype=torch.float64, device=rho.device)
        mc = material._c()
        check(lib().soptx_evaluate_general(self._h, ctypes.byref(mc), _dptr(rho, "rho", torch.float64, self.n_cells),
                                           _dptr(u, "u", torch.float64, self.ndof),
                                           _dptr(f, "f", torch.float64, self.ndof),
                                           _dptr(dc, "dc", torch.float64, self.n_cells),
                                           _dptr(c, "c", torch.float64, 2), _stream_ptr(stream)),
              "soptx_evaluate_general")
        return dc, c

    def apply_dirichlet(self, mask, K, stream=None):
        """K[r,:] = K[:,r] = 0, K[r,r] = 1 for every fixed dof r of mask, in place."""
        import torch
        check(lib().soptx_apply_dirichlet(self._h, _dptr(mask, "mask", torch.uint8, self.ndof),
                                          _dptr(K, "K", torch.float64, self.nnz), _stream_ptr(stream)),
              "soptx_apply_dirichlet")
        return K

    def sensitivity(self, material: Material, rho, u, out=None, prec: int = FP64, stream=None):
        """dc_e = -E'(rho_e) u_e^T K_e^0 u_e (Appendix D)."""
        import torch
        if out is None:
            with _on(stream):
                out = torch.empty(self.n_cells, dtype=self._rho_dtype(prec), device=rho.device)
        mc = material._c()
        check(lib().soptx_sensitivity(self._h, ctypes.byref(mc),
                                      _dptr(rho, "rho", self._rho_dtype(prec), self.n_cells),
                                      _dptr(u, "u", torch.float64, self.ndof),
                                      _dptr(out, "dc", self._rho_dtype(prec), self.n_cells), prec,
                                      _stream_ptr(stream)), "soptx_sensitivity")
        return out

    def compliance(self, material: Material, rho, u, f=None, out=None, prec: int = FP64, stream=None):
        """[u^T K u, f^T u] as a device FP64 tensor of 2 (Eq. cmpd)."""
        import torch
        if out is None:
            with _on(stream):
                out = torch.zeros(2, dtype=torch.float64, device=rho.device)
        mc = material._c()
        check(lib().soptx_compliance(self._h, ctypes.byref(mc),
                                     _dptr(rho, "rho", self._rho_dtype(prec), self.n_cells),
                                     _dptr(u, "u", torch.float64, self.ndof),
                                     _dptr(f, "f", torch.float64, self.ndof),
                                     _dptr(out, "c", torch.float64, 2), prec, _stream_ptr(stream)),
              "soptx_compliance")
        return out

    def evaluate(self, material: Material, rho, u, f=None, dc=None, c=None, prec: int = FP64, stream=None):
        """Fused sensitivity + compliance; returns (dc, c)."""
        import torch
        if dc is None:
            with _on(stream):
                dc = torch.empty(self.n_cells, dtype=self._rho_dtype(prec), device=rho.device)
        if c is None:
            with _on(stream):
                c = torch.zeros(2, dtype=torch.float64, device=rho.device)
        mc = material._c()
        check(lib().soptx_evaluate(self._h, ctypes.byref(mc),
                                   _dptr(rho, "rho", self._rho_dtype(prec), self.n_cells),
                                   _dptr(u, "u", torch.float64, self.ndof), _dptr(f, "f", torch.float64, self.ndof),
                                   _dptr(dc, "dc", self._rho_dtype(prec), self.n_cells),
                                   _dptr(c, "c", torch.float64, 2), prec, _stream_ptr(stream)), "soptx_evaluate")
        return dc, c

    def step(self, material: Material, rho, u=None, f=None, bc: Optional["Dirichlet"] = None, K=None, dc=None,
             c=None, prec: int = FP64, stream=None, want_dc: bool = True, want_c: bool = True):
        """The whole step in one pass (soptx_step): K (FP64, with the Dirichlet
        rows and columns of bc) and, when u is given, dc and c = [u^T K u, f^T u].
        Returns (K, dc, c) (dc, c None without u or when not wanted)."""
        import torch
        with _on(stream):
            if K is None:
                K = torch.empty(self.nnz, dtype=torch.float64, device=rho.device)
            if u is not None and dc is None and want_dc:
                dc = torch.empty(self.n_cells, dtype=self._rho_dtype(prec), device=rho.device)
            if u is not None and c is None and want_c:
                c = torch.empty(2, dtype=torch.float64, device=rho.device)
        mc = material._c()
        check(lib().soptx_step(self._h, None if bc is None else bc._h, ctypes.byref(mc),
                               _dptr(rho, "rho", self._rho_dtype(prec), self.n_cells),
                               _dptr(u, "u", torch.float64, self.ndof), _dptr(f, "f", torch.float64, self.ndof),
                               _dptr(K, "K", torch.float64, self.nnz),
                               _dptr(dc, "dc", self._rho_dtype(prec), self.n_cells),
                               _dptr(c, "c", torch.float64, 2), prec, _stream_ptr(stream)), "soptx_step")
        return K, dc, c

    def spmv(self, K, x, out=None, stream=None):
        """y = K x on the pattern (FP64)."""
        import torch
        if out is None:
            with _on(stream):
                out = torch.empty(self.ndof, dtype=torch.float64, device=x.device)
        check(lib().soptx_spmv(self._h, _dptr(K, "K", torch.float64, self.nnz), _dptr(x, "x", torch.float64, self.ndof),
                               _dptr(out, "y", torch.float64, self.ndof), _stream_ptr(stream)), "soptx_spmv")
        return out

    def pcg(self, K, f, u=None, rtol: float = 1e-10, max_iter: int = 10000, stream=None):
        """Solve K u = f by CG preconditioned with the nodes' diagonal blocks (K
        SPD: assembled with a Dirichlet mask).  u: initial guess, overwritten
        (zeros if None).  Stops at ||r_k|| <= rtol ||f||.
        Returns (u, iterations, ||r_k|| / ||f||)."""
        import torch
        if u is None:
            with _on(stream):
                u = torch.zeros(self.ndof, dtype=torch.float64, device=f.device)
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        check(lib().soptx_pcg(self._h, _dptr(K, "K", torch.float64, self.nnz), _dptr(f, "f", torch.float64, self.ndof),
                              _dptr(u, "u", torch.float64, self.ndof), float(rtol), int(max_iter), ctypes.byref(it),
                              ctypes.byref(rel), _stream_ptr(stream)), "soptx_pcg")
        return u, it.value, rel.value

    def backward(self, material: Material, rho, Kbar, mask=None, out=None, prec: int = FP64, stream=None):
        """drho_e = E'(rho_e) <Kbar, K_e^0> over the element's slots (reverse of assemble)."""
        import torch
        if out is None:
            with _on(stream):
                out = torch.empty(self.n_cells, dtype=self._rho_dtype(prec), device=rho.device)
        mc = material._c()
        check(lib().soptx_assemble_backward(self._h, ctypes.byref(mc),
                                            _dptr(rho, "rho", self._rho_dtype(prec), self.n_cells),
                                            _dptr(mask, "mask", torch.uint8, self.ndof),
                                            _dptr(Kbar, "Kbar", torch.float64, self.nnz),
                                            _dptr(out, "drho", self._rho_dtype(prec), self.n_cells), prec,
                                            _stream_ptr(stream)), "soptx_assemble_backward")
        return out


class Dirichlet:
    """Dirichlet rows and columns bound once to a pattern (soptx_build_dirichlet):
    mask is a host array of ndof uint8, nonzero = fixed dof.  Used by
    Pattern.step; close it (or let it be collected) before the pattern."""

    def __init__(self, pattern: Pattern, mask, stream=None):
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.shape != (pattern.ndof,):
            raise ValueError(f"mask must have {pattern.ndof} entries")
        h = ctypes.c_void_p()
        check(lib().soptx_build_dirichlet(pattern._h, mask.ctypes.data, ctypes.byref(h), _stream_ptr(stream)),
              "soptx_build_dirichlet")
        self._h = h
        self._pattern = pattern   # keeps the pattern alive while the table exists
        nf, ng = ctypes.c_int64(), ctypes.c_int64()
        check(lib().soptx_dirichlet_info(h, ctypes.byref(nf), ctypes.byref(ng)), "soptx_dirichlet_info")
        self.n_fixed, self.n_groups = nf.value, ng.value

    def close(self):
        if getattr(self, "_h", None):
            lib().soptx_destroy_dirichlet(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def filter_stencil_host(elem: int, coords, cells, rmin: float):
    """(offsets, grid sizes) of the stencil form soptx_build_filter_ex would use
    for this mesh and radius; (0, (0, 0, 0)) when it would use the CSR form."""
    m, keep = _mesh_struct(elem, coords, cells)
    S = ctypes.c_int32()
    N = (ctypes.c_int64 * 3)()
    check(lib().soptx_debug_filter_stencil(ctypes.byref(m), float(rmin), ctypes.byref(S), N),
          "soptx_debug_filter_stencil")
    return S.value, tuple(N)


def filter_matrix_host(elem: int, coords, cells, rmin: float) -> dict:
    """The filter matrix soptx_build_filter uploads, built on the host only:
    row_ptr, col, w, element measures vol, row sums hsv (H v) and hs (H 1)."""
    m, keep = _mesh_struct(elem, coords, cells)
    n, nnz = ctypes.c_int64(), ctypes.c_int64()
    check(lib().soptx_debug_filter_matrix(ctypes.byref(m), float(rmin), ctypes.byref(n), ctypes.byref(nnz),
                                          None, None, None, None, None, None), "soptx_debug_filter_matrix")
    out = {"row_ptr": np.zeros(n.value + 1, np.int32), "col": np.zeros(max(nnz.value, 1), np.int32),
           "w": np.zeros(max(nnz.value, 1)), "vol": np.zeros(max(n.value, 1)), "hsv": np.zeros(max(n.value, 1)),
           "hs": np.zeros(max(n.value, 1))}
    check(lib().soptx_debug_filter_matrix(ctypes.byref(m), float(rmin), ctypes.byref(n), ctypes.byref(nnz),
                                          *(out[k].ctypes.data for k in ("row_ptr", "col", "w", "vol", "hsv", "hs"))),
          "soptx_debug_filter_matrix")
    for k in ("col", "w"):
        out[k] = out[k][: nnz.value]
    for k in ("vol", "hsv", "hs"):
        out[k] = out[k][: n.value]
    return out


class Filter:
    """The filter matrix H of a mesh (Sec. 2.4), resident on the device:
    H_ij = max(0, rmin - dist(i, j)) over element centroids, built once per
    mesh; the sensitivity filter, the density filter with the Heaviside
    projection, and the density filter's chain rule run per call (FP64)."""

    def __init__(self, elem: int, coords, cells, rmin: float, csr_only: bool = False, stream=None):
        m, keep = _mesh_struct(elem, coords, cells)
        h = ctypes.c_void_p()
        check(lib().soptx_build_filter_ex(ctypes.byref(m), float(rmin), _lib.FILTER_CSR_ONLY if csr_only else 0,
                                          ctypes.byref(h), _stream_ptr(stream)), "soptx_build_filter")
        self._h = h
        self.rmin = float(rmin)
        n, nnz, rpb, S = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().soptx_filter_info(h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(rpb)), "filter_info")
        check(lib().soptx_filter_stencil_size(h, ctypes.byref(S)), "filter_stencil_size")
        self.n, self.nnz, self.rows_per_block = n.value, nnz.value, rpb.value
        self.stencil_size = S.value        # offsets of the stencil form (0: CSR form)

    @classmethod
    def from_mesh(cls, mesh, rmin: float, **kw) -> "Filter":
        return cls(mesh.elem, mesh.coords, mesh.cells, rmin, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().soptx_destroy_filter(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matrix(self):
        """(row_ptr int32, col int32, w float64, element measures float64) on the host."""
        rp = np.zeros(self.n + 1, dtype=np.int32)
        col = np.zeros(max(self.nnz, 1), dtype=np.int32)
        w = np.zeros(max(self.nnz, 1))
        v = np.zeros(max(self.n, 1))
        check(lib().soptx_filter_copy(self._h, rp.ctypes.data, col.ctypes.data, w.ctypes.data, v.ctypes.data),
              "soptx_filter_copy")
        return rp, col[: self.nnz], w[: self.nnz], v[: self.n]

    def volumes(self):
        """The element measures v (float64, host)."""
        v = np.zeros(max(self.n, 1))
        check(lib().soptx_filter_copy(self._h, None, None, None, v.ctypes.data), "soptx_filter_copy")
        return v[: self.n]

    def sensitivity(self, rho, dc, out=None, stream=None):
        """dc~_i = sum_j H_ij rho_j dc_j / (max(1e-3, rho_i) sum_j H_ij)."""
        import torch
        if out is None:
            with _on(stream):
                out = torch.empty(self.n, dtype=torch.float64, device=rho.device)
        check(lib().soptx_filter_sensitivity(self._h, _dptr(rho, "rho", torch.float64, self.n),
                                             _dptr(dc, "dc", torch.float64, self.n),
                                             _dptr(out, "dc_out", torch.float64, self.n), _stream_ptr(stream)),
              "soptx_filter_sensitivity")
        return out

    def density(self, rho, beta: Optional[float] = None, rho_tilde=None, rho_bar=None, stream=None):
        """rho~ = (H (v rho)) / (H v); with beta, also the Heaviside projection
        rho_bar = 1 - exp(-beta rho~) + rho~ exp(-beta).  Returns rho~, or
        (rho~, rho_bar) with beta."""
        import torch
        if rho_tilde is None:
            with _on(stream):
                rho_tilde = torch.empty(self.n, dtype=torch.float64, device=rho.device)
        if beta is not None and rho_bar is None:
            with _on(stream):
                rho_bar = torch.empty(self.n, dtype=torch.float64, device=rho.device)
        check(lib().soptx_filter_density(self._h, _dptr(rho, "rho", torch.float64, self.n),
                                         float(beta if beta is not None else 0.0),
                                         _dptr(rho_tilde, "rho_tilde", torch.float64, self.n),
                                         _dptr(rho_bar, "rho_bar", torch.float64, self.n) if beta is not None else None,
                                         _stream_ptr(stream)), "soptx_filter_density")
        return rho_tilde if beta is None else (rho_tilde, rho_bar)

    def density_backward(self, grad, rho_tilde=None, beta: Optional[float] = None, out=None, stream=None):
        """dpsi/drho from dpsi/drho~ (rho_tilde None), or from dpsi/drho_bar
        through the Heaviside projection at beta and rho_tilde."""
        import torch
        if (rho_tilde is None) != (beta is None):
            raise ValueError("rho_tilde and beta go together")
        if out is None:
            with _on(stream):
                out = torch.empty(self.n, dtype=torch.float64, device=grad.device)
        check(lib().soptx_filter_density_backward(
            self._h, _dptr(rho_tilde, "rho_tilde", torch.float64, self.n), float(beta if beta is not None else 0.0),
            _dptr(grad, "grad", torch.float64, self.n), _dptr(out, "grad_rho", torch.float64, self.n),
            _stream_ptr(stream)), "soptx_filter_density_backward")
        return out


def heaviside_beta(iteration: int, beta0: float = 1.0, max_beta: float = 512.0, every: int = 50) -> float:
    """Continuation of the projection parameter: beta0 doubled every `every`
    iterations, capped at max_beta (Sec. 5.2 uses 1, 512 and 50)."""
    if iteration < 0 or every <= 0:
        raise ValueError("iteration >= 0 and every > 0")
    beta = float(beta0)
    for _ in range(iteration // every):
        if beta >= max_beta:
            break
        beta *= 2.0
    return float(min(max_beta, beta))


def oc_update(rho, dc, dv, vol_target: float, move: float = 0.2, eta: float = 0.5, lmax: float = 1e9,
              tol: float = 1e-3, max_steps: int = 200, out=None, stream=None):
    """One optimality-criteria update (Sec. 2.3): rho_new = rho B^eta clamped by
    the move limit, B = max(0, -dc) / (lambda dv), lambda by bisection so that
    sum dv rho_new = vol_target.  Returns (rho_new, {lambda, volume, change, steps})."""
    import torch
    n = int(rho.numel())
    if out is None:
        with _on(stream):
            out = torch.empty(n, dtype=torch.float64, device=rho.device)
    prm = _lib.OcParams(float(move), float(eta), float(lmax), float(tol), int(max_steps))
    res = _lib.OcResult()
    check(lib().soptx_oc_update(n, _dptr(rho, "rho", torch.float64, n), _dptr(dc, "dc", torch.float64, n),
                                _dptr(dv, "dv", torch.float64, n), float(vol_target), ctypes.byref(prm),
                                _dptr(out, "rho_new", torch.float64, n), ctypes.byref(res), _stream_ptr(stream)),
          "soptx_oc_update")
    return out, {"lambda": res.lambda_, "volume": res.volume, "change": res.change, "steps": res.steps}
