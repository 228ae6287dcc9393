"""CPU tests of the HIP library's host side (no device work).

* the shared library loads and exports every function include/*.h declares;
* mesh validation error paths;
* the reference tensor against exact rational integrals (tests/exact_fe.py);
* the host pattern is bit-identical to the oracle's set-based pattern;
* the assembly plan is complete and consistent (every element-local pair
  (e, i, j) lands exactly once, in the right row, column and order), and a
  numpy model that walks the plan with the separated element formula matches
  the oracle's standard-quadrature assembly.
"""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import exact_fe
from oracle import oracle as O
from paper_2505_02438_amd import _lib, api
from paper_2505_02438_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ELEMS = [I.QUAD4, I.TRI3, I.HEX8, I.TET10]


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(soptx_\w+)\s*\(", txt):
            names.add(m.group(1))
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(L, n), n


def test_status_strings():
    L = _lib.lib()
    for code in range(0, -10, -1):
        assert L.soptx_status_string(code)
    assert L.soptx_status_string(-99) == b"unknown status"


def _bad(elem, coords, cells):
    return api.validate_mesh(elem, coords, cells)


def test_validation_error_codes():
    m = I.quad_grid(3, 2)
    assert _bad(m.elem, m.coords, m.cells) == 0
    c = m.cells.copy()
    c[1, 2] = m.n_nodes  # out of range
    assert _bad(m.elem, m.coords, c) == -3
    c = m.cells.copy()
    c[1, 2] = c[1, 0]  # repeated node
    assert _bad(m.elem, m.coords, c) == -3
    c = m.cells[:, ::-1].copy()  # clockwise: inverted
    assert _bad(m.elem, m.coords, c) == -4
    x = m.coords.copy()
    x[5] += [0.1, 0.05]  # interior node moved: quads no longer parallelograms
    assert _bad(m.elem, x, m.cells) == -5
    assert _bad(9, m.coords, m.cells) == -2
    # hexes and P2 tets
    h = I.hex_grid(2, 2, 2)
    xh = h.coords.copy()
    xh[13] += 0.1
    assert _bad(h.elem, xh, h.cells) == -5
    t = I.kuhn_p2_tets(2, 1, 1)
    xt = t.coords.copy()
    edge_node = t.cells[0, 5]
    xt[edge_node] += 0.05  # curved edge
    assert _bad(t.elem, xt, t.cells) == -5
    # null pointers / wrong dim through the raw ABI
    L = _lib.lib()
    mesh = _lib.Mesh(I.QUAD4, 2, m.n_nodes, None, m.n_cells, None)
    assert L.soptx_validate_mesh(ctypes.byref(mesh)) == -1
    mesh = _lib.Mesh(I.QUAD4, 3, m.n_nodes, m.coords.ctypes.data, m.n_cells, m.cells.ctypes.data)
    assert L.soptx_validate_mesh(ctypes.byref(mesh)) == -1
    assert L.soptx_validate_mesh(None) == -1


def test_debug_variant_hooks_check_their_arguments():
    """The process-wide variant hooks accept only their listed values, and
    the general-path query refuses a null handle or output, with no device
    work."""
    L = _lib.lib()
    try:
        for v in (-1, 0, 1):
            assert L.soptx_debug_set_assembly_variant(v) == 0
            assert L.soptx_debug_set_general_variant(v) == 0
        for v in (-2, 2, 7):
            assert L.soptx_debug_set_assembly_variant(v) == -1
            assert L.soptx_debug_set_general_variant(v) == -1
    finally:
        L.soptx_debug_set_assembly_variant(-1)
        L.soptx_debug_set_general_variant(-1)
    form = ctypes.c_int32(5)
    assert L.soptx_debug_general_path(None, ctypes.byref(form)) == -1
    assert form.value == 5


def test_per_call_argument_errors_without_device():
    """Calls with a NULL handle or bad arguments fail before any device work."""
    L = _lib.lib()
    mat = _lib.Material(1.0, 1e-9, 0.3, 3.0, 0)
    assert L.soptx_assemble(None, ctypes.byref(mat), None, None, None, 0, None) == -1
    assert L.soptx_sensitivity(None, ctypes.byref(mat), None, None, None, 0, None) == -1
    assert L.soptx_compliance(None, ctypes.byref(mat), None, None, None, None, 0, None) == -1
    assert L.soptx_evaluate(None, ctypes.byref(mat), None, None, None, None, None, 0, None) == -1
    assert L.soptx_assemble_backward(None, ctypes.byref(mat), None, None, None, None, 0, None) == -1
    assert L.soptx_apply_dirichlet(None, None, None, None) == -1
    assert L.soptx_spmv(None, None, None, None, None) == -1
    it, rel = ctypes.c_int32(5), ctypes.c_double(5.0)
    assert L.soptx_pcg(None, None, None, None, 1e-10, 10, ctypes.byref(it), ctypes.byref(rel), None) == -1
    assert L.soptx_pattern_info(None, None, None, None, None) == -1
    assert L.soptx_pattern_copy(None, None, None) == -1
    L.soptx_destroy_pattern(None)
    out = ctypes.c_void_p(1)
    assert L.soptx_build_pattern_ex(None, 0, ctypes.byref(out), None) == -1
    assert out.value is None
    assert L.soptx_build_pattern_ex(None, 7, ctypes.byref(out), None) == -1


@pytest.mark.parametrize("elem", ELEMS)
def test_reference_tensor_symbolic_exact(elem):
    ex = exact_fe.exact_ref_moments(elem)
    exf = np.array([[[[float(ex[i][j][m][n]) for n in range(len(ex[0][0][0]))]
                      for m in range(len(ex[0][0]))] for j in range(len(ex[0]))] for i in range(len(ex))])
    M = api.reference_tensor(elem, api.REF_SYMBOLIC)
    assert np.array_equal(M, exf)
    Mq = api.reference_tensor(elem, api.REF_QUADRATURE)
    assert np.max(np.abs(Mq - exf)) <= 8 * np.finfo(float).eps * np.max(np.abs(exf))


@pytest.mark.parametrize("elem", ELEMS)
@pytest.mark.parametrize("seed", [3, 4])
def test_host_pattern_matches_oracle(elem, seed):
    pr = I.small_problem(elem, seed=seed)
    hp = api.host_plan(elem, pr.mesh.coords, pr.mesh.cells)
    rp, ci = O.pattern(elem, pr.mesh.n_nodes, pr.mesh.cells)
    assert np.array_equal(hp["row_ptr"], rp) and np.array_equal(hp["col_idx"], ci)


def test_host_pattern_matches_oracle_configs():
    for mesh in [I.quad_grid(60, 20), I.tri_grid(60, 20, jitter=0.2, rng=np.random.default_rng(1)),
                 I.hex_grid(12, 4, 4), I.kuhn_p2_tets(4, 3, 3, jitter=0.15, rng=np.random.default_rng(2))]:
        hp = api.host_plan(mesh.elem, mesh.coords, mesh.cells)
        rp, ci = O.pattern(mesh.elem, mesh.n_nodes, mesh.cells)
        assert np.array_equal(hp["row_ptr"], rp) and np.array_equal(hp["col_idx"], ci)


def test_host_pattern_shuffled_mesh():
    rng = np.random.default_rng(5)
    m = I.kuhn_p2_tets(2, 2, 2, jitter=0.1, rng=rng)
    perm = rng.permutation(m.n_nodes)
    cells = perm[m.cells][rng.permutation(m.n_cells)].astype(np.int32)
    coords = np.empty_like(m.coords)
    coords[perm] = m.coords
    hp = api.host_plan(m.elem, coords, cells)
    rp, ci = O.pattern(m.elem, m.n_nodes, cells)
    assert np.array_equal(hp["row_ptr"], rp) and np.array_equal(hp["col_idx"], ci)


def _lame(dim, nu, plane_strain=0):
    mu = 1.0 / (2.0 * (1.0 + nu))
    lam = nu / (1.0 - nu * nu) if (dim == 2 and not plane_strain) else nu / ((1 + nu) * (1 - 2 * nu))
    return lam, mu


def walk_plan(hp, mesh, rho, M, E0=1.0, Emin=1e-9, p=3.0, nu=0.3, mask=None):
    """Model of the assembly kernel's walk over the plan (numpy, FP64)."""
    D, nen, NC = mesh.dim, mesh.nen, mesh.n_cells
    cells = mesh.cells
    geo = hp["geo"].reshape(D * D + 1, NC)
    G = geo[: D * D].T.reshape(NC, D, D)
    det = geo[D * D]
    E = Emin + rho ** p * (E0 - Emin)
    Gp = np.sqrt(E * det)[:, None, None] * G
    lam, mu = _lame(D, nu)
    rp, ci = hp["row_ptr"], hp["col_idx"]
    K = np.full(hp["nnz"], np.nan)
    seen = np.zeros((NC, nen, nen), dtype=np.int32)
    gi = hp["grp_info"].reshape(-1, 6)
    si = hp["sig_info"].reshape(-1, 4)
    NG = hp["grp_nodes"].size // gi.shape[0]  # nodes per group (slots of the node tables)
    assert NG == 32
    for g in range(gi.shape[0]):
        sig, nn, eoff, ne, n2loff, flags = gi[g]
        Kk, deg, posoff, blk = si[sig]
        assert blk % 2 == 1 and blk >= D * D * deg
        cnt = np.diff(hp["sig_pos_ptr"][posoff:posoff + deg + 1])
        items = hp["sig_pairs"][2 * posoff:2 * posoff + 2 * (deg + 1)].reshape(deg + 1, 2)
        nit = int(np.argmax(items[:, 0] < 0))
        assert np.all(items[nit:] == -1)
        split = {}  # position -> number of contributions taken by the low half
        covered = []
        costs = []
        for pa, pb in items[:nit]:
            assert pa >= 0
            if pb == pa:
                split[pa] = (cnt[pa] + 1) // 2
                covered.append(pa)
                costs.append((cnt[pa] + 1) // 2)
            else:
                covered += [pa] + ([pb] if pb >= 0 else [])
                assert pb < 0 or cnt[pa] >= cnt[pb]  # the low half runs the longer list
                costs.append(cnt[pa])
        assert sorted(covered) == list(range(deg))  # every position exactly once
        # the pair path reads codes in chunks of 8, both halves as many chunks
        # as the low (longer) list needs: every such read stays in the table
        ncodes = hp["sig_contrib"].size
        pos = hp["sig_pos_ptr"]
        for pa, pb in items[:nit]:
            c0, na = int(pos[posoff + pa]), int(cnt[pa])
            lo0, nlo, hi0, nhi = c0, na, c0, 0
            if pb == pa:
                nlo = (na + 1) // 2
                hi0, nhi = c0 + nlo, na - nlo
            elif pb >= 0:
                hi0, nhi = int(pos[posoff + pb]), int(cnt[pb])
            span = -(-nlo // 8) * 8
            assert lo0 + span <= ncodes and (hi0 if nhi > 0 else lo0) + span <= ncodes
        assert np.all(np.diff(costs) <= 0)  # costliest first
        wsh = (flags >> 1) & 3
        if wsh:
            # wide work items: P positions x Q phases x N nodes = 64 lanes
            N = 32 >> wsh
            assert nn <= N
            wr = hp["sig_witems"].reshape(-1, 32)[hp["sig_witem_ptr"][sig]:hp["sig_witem_ptr"][sig + 1]]
            wcov, wcost = [], []
            for rec in wr:
                P, Q, T = (int(x) for x in rec[:3])
                assert Q & (Q - 1) == 0 and 1 <= P and P * Q * N <= 64 and T <= 8
                tmax = 0
                for k in range(8):
                    p, off, c = int(rec[8 + k]), int(rec[16 + k]), int(rec[24 + k])
                    if k < P:
                        assert off == hp["sig_pos_ptr"][posoff + p] and c == cnt[p]
                        wcov.append(p)
                        tmax = max(tmax, -(-c // Q))
                    else:
                        assert p == -1 and c == 0
                assert T == tmax
                wcost.append(T)
            assert sorted(wcov) == list(range(deg)) and np.all(np.diff(wcost) <= 0)
            split = {}  # the phases of a position are summed by the kernel's butterfly
        else:
            assert hp["sig_witem_ptr"][sig + 1] == hp["sig_witem_ptr"][sig]
        elems = hp["grp_elems"][eoff:eoff + ne]
        # canonical-order plans: elements listed by rank (ascending), a rank
        # table per group
        ro = int(hp["grp_rank_off"][g]) if hp["grp_rank_off"].size else -1
        canon = hp["grp_rank_off"].size > 0
        if canon:
            assert np.all(np.diff(elems) > 0)
            elems = hp["elem_by_rank"][elems]
        assert ne <= hp["emax"] and len(np.unique(elems)) == ne and (canon or np.all(np.diff(elems) > 0))
        offdiag = G[elems][:, ~np.eye(D, dtype=bool)]
        assert (flags & 1) == (1 if np.all(offdiag == 0.0) else 0)
        n2l = hp["grp_n2l"][n2loff:n2loff + Kk * NG].reshape(Kk, NG)
        for lane in range(nn):
            Inode = hp["grp_nodes"][NG * g + lane]
            base = rp[D * Inode]
            rowlen = rp[D * Inode + 1] - base
            assert hp["grp_rows"][2 * NG * g + 2 * lane] == base and hp["grp_rows"][2 * NG * g + 2 * lane + 1] == rowlen
            assert rowlen == D * deg
            prev_e = None
            for pp in range(deg):
                c0, c1 = hp["sig_pos_ptr"][posoff + pp], hp["sig_pos_ptr"][posoff + pp + 1]
                parts = [np.zeros((D, D)), np.zeros((D, D))]
                last = -1
                pc = int(hp["grp_rank"][ro + pp * NG + lane]) if ro >= 0 else pp  # CSR position
                Jcol = ci[base + D * pc] // D
                for t in range(c0, c1):
                    pk = int(hp["sig_contrib"][t])
                    k, i, j = pk >> 16, (pk >> 8) & 255, pk & 255
                    e = elems[n2l[k, lane]]
                    assert cells[e, i] == Inode and cells[e, j] == Jcol
                    assert canon or e > last  # ascending elements within a stored block
                    last = e
                    seen[e, i, j] += 1
                    half = 1 if pp in split and t - c0 >= split[pp] else 0
                    parts[half] += Gp[e].T @ M[i, j] @ Gp[e]
                acc = parts[0] + parts[1]  # a split position: low half's sum + high half's
                out = lam * acc + mu * acc.T + mu * np.trace(acc) * np.eye(D)
                if mask is not None:
                    for a in range(D):
                        for b in range(D):
                            r, c = D * Inode + a, D * Jcol + b
                            if mask[r] or mask[c]:
                                out[a, b] = 1.0 if r == c else 0.0
                for a in range(D):
                    K[base + a * rowlen + D * pc: base + a * rowlen + D * pc + D] = out[a]
    assert np.all(seen == 1), "every element-local pair must be assembled exactly once"
    return K


def row_scaled_err(rp, Kx, Kref):
    """max over rows of max|dK| / max|Kref| in the row (structural cancellations kept)."""
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    den = np.zeros(n)
    np.maximum.at(den, rows, np.abs(Kref))
    num = np.zeros(n)
    np.maximum.at(num, rows, np.abs(Kx - Kref))
    ok = den > 0
    return float(np.max(num[ok] / den[ok])) if ok.any() else 0.0


@pytest.mark.parametrize("elem", ELEMS)
@pytest.mark.parametrize("use_mask", [False, True])
def test_plan_walk_model_matches_oracle(elem, use_mask):
    pr = I.small_problem(elem, seed=6)
    m = pr.mesh
    hp = api.host_plan(elem, m.coords, m.cells)
    M = api.reference_tensor(elem)
    mask = pr.mask if use_mask else None
    K = walk_plan(hp, m, pr.rho, M, mask=mask)
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    Kref = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci, mask=mask)
    assert not np.isnan(K).any()
    assert row_scaled_err(rp, K, Kref) <= 1e-13


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8])
@pytest.mark.parametrize("skew", ["global", "kink"])
def test_plan_walk_skewed_q1(elem, skew):
    """Sheared Q1 meshes: the axis-aligned flag is off for every group ('global')
    or for the groups that touch the sheared half ('kink')."""
    pr = I.small_problem(elem, seed=6, skew=skew, dims=(8, 5) if elem == I.QUAD4 else (6, 4, 5))
    m = pr.mesh
    hp = api.host_plan(elem, m.coords, m.cells)
    flags = hp["grp_info"].reshape(-1, 6)[:, 5] & 1  # bit 0: axis-aligned
    if skew == "global":
        assert np.all(flags == 0)
    else:
        assert np.any(flags == 1) and np.any(flags == 0)
    K = walk_plan(hp, m, pr.rho, api.reference_tensor(elem), mask=pr.mask)
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    Kref = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci, mask=pr.mask)
    assert row_scaled_err(rp, K, Kref) <= 1e-13


def _renumbered(mesh, seed):
    rng = np.random.default_rng(seed)
    pn = rng.permutation(mesh.n_nodes)       # new id of old node i: pn[i]
    pe = rng.permutation(mesh.n_cells)       # old element of new element k: pe[k]
    coords = np.empty_like(mesh.coords)
    coords[pn] = mesh.coords
    return I.Mesh(mesh.elem, coords, pn[mesh.cells[pe]].astype(np.int32)), pn, pe


@pytest.mark.parametrize("elem,dims", [(I.QUAD4, (12, 7)), (I.HEX8, (9, 6, 5)), (I.TRI3, (9, 6)), (I.TET10, (4, 3, 3))])
def test_plan_survives_renumbering(elem, dims):
    """Nodes and elements renumbered by a seeded permutation: the plan takes
    the canonical order, so it has the signatures and group sizes of the
    lexicographically numbered mesh (a rank table per group maps canonical
    positions to CSR columns), and its walk still gives the oracle's K."""
    pr = I.small_problem(elem, seed=6, jitter=False, dims=dims)
    m0 = pr.mesh
    hp0 = api.host_plan(elem, m0.coords, m0.cells)
    m, pn, pe = _renumbered(m0, 91)
    hp = api.host_plan(elem, m.coords, m.cells)
    assert hp["grp_rank_off"].size == hp["n_groups"] and np.any(hp["grp_rank_off"] >= 0)
    assert hp0["grp_rank_off"].size == 0          # numbered along the grid: the given numbering is kept
    assert hp["n_signatures"] <= hp0["n_signatures"]
    sizes = lambda h: sorted(h["grp_info"].reshape(-1, 6)[:, 1].tolist())
    assert sizes(hp) == sizes(hp0)
    rho = pr.rho[pe]
    mask = np.empty_like(pr.mask)
    mask.reshape(-1, m.dim)[pn] = pr.mask.reshape(-1, m.dim)
    M = api.reference_tensor(elem)
    rp, ci = O.pattern(elem, m.n_nodes, m.cells)
    for msk in (None, mask):
        K = walk_plan(hp, m, rho, M, mask=msk)
        Kref = O.assemble(elem, m.coords, m.cells, rho, rp, ci, mask=msk)
        assert not np.isnan(K).any()
        assert row_scaled_err(rp, K, Kref) <= 1e-13


def test_grid_numbered_meshes_keep_their_numbering():
    """Meshes numbered along the grid (the generators' numberings) have few
    signatures already: the plan keeps the given order (no rank tables)."""
    for m in [I.quad_grid(9, 4), I.hex_grid(5, 3, 4), I.skew_mesh(I.hex_grid(4, 3, 3), "global")]:
        hp = api.host_plan(m.elem, m.coords, m.cells)
        assert hp["grp_rank_off"].size == 0


def test_plan_axis_aligned_flag_set_on_grids():
    for mesh in [I.quad_grid(9, 4), I.hex_grid(5, 3, 4)]:
        hp = api.host_plan(mesh.elem, mesh.coords, mesh.cells)
        assert np.all(hp["grp_info"].reshape(-1, 6)[:, 5] & 1 == 1)


@pytest.mark.parametrize("elem", ELEMS)
def test_transposed_slot_table(elem):
    """For node n and neighbour J = nb(n)[q]: nb_tslot = CSR slot of
    (row dim J, column dim n), nb_tdeg = degree of J (used to reach the column
    entries of a fixed dof)."""
    pr = I.small_problem(elem, seed=5)
    m = pr.mesh
    hp = api.host_plan(elem, m.coords, m.cells)
    D = m.dim
    rp, ci = hp["row_ptr"], hp["col_idx"]
    nbrs = [ci[rp[D * n]:rp[D * n + 1]:D] // D for n in range(m.n_nodes)]
    ptr = np.concatenate([[0], np.cumsum([len(x) for x in nbrs])])
    assert hp["nb_tslot"].size == ptr[-1] and hp["nb_tdeg"].size == ptr[-1]
    for n in range(m.n_nodes):
        assert rp[D * n] == D * D * ptr[n]
        for q, J in enumerate(nbrs[n]):
            k = ptr[n] + q
            t = hp["nb_tslot"][k]
            assert hp["nb_tdeg"][k] == len(nbrs[J])
            assert rp[D * J] <= t < rp[D * J + 1] and ci[t] == D * n  # row D J, column D n
            assert (t == rp[D * n] + D * q) == (J == n)  # the kernel's test for J == n


def test_backward_position_table():
    pr = I.small_problem(I.TET10, seed=2)
    m = pr.mesh
    hp = api.host_plan(m.elem, m.coords, m.cells)
    pos = hp["pos"].reshape(m.n_cells, m.nen, m.nen)
    rp, ci = hp["row_ptr"], hp["col_idx"]
    D = m.dim
    for e in range(m.n_cells):
        for i in range(m.nen):
            for j in range(m.nen):
                Inode, Jnode = m.cells[e, i], m.cells[e, j]
                assert ci[rp[D * Inode] + D * pos[e, i, j]] == D * Jnode


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8, I.TET10])
def test_dirichlet_slot_walk_matches_oracle(elem):
    """The Dirichlet kernel's write set, walked on the host from the plan tables
    (lane per fixed dof r = D n + a; for each neighbour J = nb(n)[q] it writes
    row r's D slots at rp[r] + D q + e and column r's D slots at
    nb_tslot + e D deg(J) + a), gives the oracle's K with fixed rows and columns
    replaced by identity ones."""
    pr = I.small_problem(elem, seed=17)
    m = pr.mesh
    hp = api.host_plan(elem, m.coords, m.cells)
    D = m.dim
    rp, ci = hp["row_ptr"], hp["col_idx"]
    K = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci)
    ref = O.assemble(elem, m.coords, m.cells, pr.rho, rp, ci, mask=pr.mask)
    Kw = K.copy()
    ts_all, td_all = hp["nb_tslot"].astype(np.int64), hp["nb_tdeg"].astype(np.int64)
    for r in np.flatnonzero(pr.mask):
        n, a = divmod(int(r), D)
        ib = int(rp[D * n])
        deg = (int(rp[r + 1]) - int(rp[r])) // D
        nptr = ib // (D * D)
        for q in range(deg):
            ts, jl = int(ts_all[nptr + q]), D * int(td_all[nptr + q])
            self_ = ts == ib + D * q
            for e in range(D):
                v = 1.0 if (self_ and e == a) else 0.0
                i_row, i_col = int(rp[r]) + D * q + e, ts + e * jl + a
                assert 0 <= i_row < ci.size and 0 <= i_col < ci.size
                assert ci[i_row] == D * int(ci[ib + D * q] // D) + e and ci[i_col] == r
                Kw[i_row] = v
                Kw[i_col] = v
    assert np.array_equal(Kw, ref)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU's share: --gpus above 1 exits with a message
    before touching a device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and msg["n_gpus"] == 2


def _raw_host_plan(m):
    """Status of the host build (pattern + plan) of a mesh through the raw ABI."""
    L = _lib.lib()
    mesh, keep = api._mesh_struct(m.elem, m.coords, m.cells)
    h = ctypes.c_void_p()
    rc = L.soptx_debug_host_plan_ex(ctypes.byref(mesh), 0, ctypes.byref(h))
    if rc == 0:
        L.soptx_debug_host_plan_free(h)
    else:
        assert h.value is None
    return rc


def test_plan_build_worker_failure_returns_oom():
    """A worker chunk that fails (forced through the test hook) makes the build
    return SOPTX_E_OOM with every thread joined; the next build succeeds."""
    L = _lib.lib()
    big = I.hex_grid(20, 20, 20)     # above the size where the build uses threads
    small = I.quad_grid(4, 3)        # built on the calling thread
    try:
        for m in (big, small):
            for n in (1, 3):
                assert L.soptx_debug_fail_workers(n) == 0
                assert _raw_host_plan(m) == -7
                assert L.soptx_debug_fail_workers(0) == 0
                assert _raw_host_plan(m) == 0
        assert L.soptx_debug_fail_workers(-1) == -1
    finally:
        L.soptx_debug_fail_workers(0)


def test_overflow_paths_before_allocation():
    """Sizes beyond the int32 index range are refused with SOPTX_E_OVERFLOW by
    the checks that run before anything is read or allocated."""
    L = _lib.lib()
    dummy_x = np.zeros(3)
    dummy_c = np.zeros(8, dtype=np.int32)
    # dof count 3 * 2^30 >= 2^31 - 1
    mesh = _lib.Mesh(I.HEX8, 3, 1 << 30, dummy_x.ctypes.data, 1, dummy_c.ctypes.data)
    assert L.soptx_validate_mesh(ctypes.byref(mesh)) == -6
    # n_cells * nen >= 2^31 - 1
    mesh = _lib.Mesh(I.HEX8, 3, 8, dummy_x.ctypes.data, (2**31 - 1) // 8, dummy_c.ctypes.data)
    assert L.soptx_validate_mesh(ctypes.byref(mesh)) == -6
    out = ctypes.c_void_p()
    assert L.soptx_debug_host_plan_ex(ctypes.byref(mesh), 0, ctypes.byref(out)) == -6


def test_adjacency_cap_overflow():
    """A node with more adjacent elements than the assembly plan's slot table
    holds (32) is refused with SOPTX_E_OVERFLOW; 32 are accepted."""
    for n, expect in ((32, 0), (33, -6)):
        ang = 2 * np.pi * np.arange(n) / n
        coords = np.vstack([[0.0, 0.0], np.stack([np.cos(ang), np.sin(ang)], axis=1)])
        cells = np.array([[0, 1 + k, 1 + (k + 1) % n] for k in range(n)], dtype=np.int32)
        m = I.Mesh(I.TRI3, coords, cells)
        assert api.validate_mesh(m.elem, m.coords, m.cells) == 0
        assert _raw_host_plan(m) == expect, n
