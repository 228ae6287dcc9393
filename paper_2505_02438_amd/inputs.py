"""Seeded synthetic inputs: meshes, boundary masks, loads, densities, displacements.

This module holds no finite-element arithmetic.  It only lays out geometry and
draws random numbers, and it is shared by the HIP path's tests/bench and the
CPU oracle's tests so that both sides see identical arrays.

Conventions (inputs to both sides, so they are not parity questions):

* Degrees of freedom are interleaved node-major: ``dof = dim * node + comp``
  (the vector Lagrange space of Section 4.2 with shape ``(-1, dim)``).
* Structured node ids put x slowest: 2D ``i*(ny+1)+j``; 3D
  ``(i*(ny+1)+j)*(nz+1)+k``.  Element ids follow the same order.
* Local node orders:
    - Q1 quad: (0,0),(1,0),(1,1),(0,1), counter-clockwise.
    - Q1 hex: bottom face counter-clockwise, then top face counter-clockwise.
    - P1 triangle: counter-clockwise.  Each square (i,j) is split along its
      (i,j)-(i+1,j+1) diagonal.
    - P2 tetrahedron: 4 positively oriented vertices, then the edge nodes of
      edges 01, 02, 03, 12, 13, 23.  Cubes are split into the 6 Kuhn
      (Freudenthal) tetrahedra along the (0,0,0)-(1,1,1) diagonal.
* Jitter moves interior *vertices* only; P2 edge nodes sit at the midpoints
  of the (straight) jittered edges, so every element stays affine.

Boundary conditions and loads follow the problem definitions of Appendices
A-C (Cantilever2dData1, MBBBeam2dData1, Cantilever3dData1): zero Dirichlet
values, nodal point loads placed straight into f.

Seeds: configuration k draws from ``numpy.random.default_rng(1000 + k)``;
serving request r from ``default_rng(5000 + r)``.  Draw order is jitter,
then densities, then displacements.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# element type codes shared with the C ABI (see include/soptx.h)
QUAD4 = 1
TRI3 = 2
HEX8 = 3
TET10 = 4
HEX27 = 5

ELEM_NAMES = {QUAD4: "quad4", TRI3: "tri3", HEX8: "hex8", TET10: "tet10", HEX27: "hex27"}
ELEM_DIM = {QUAD4: 2, TRI3: 2, HEX8: 3, TET10: 3, HEX27: 3}
ELEM_NEN = {QUAD4: 4, TRI3: 3, HEX8: 8, TET10: 10, HEX27: 27}


@dataclasses.dataclass
class Mesh:
    elem: int
    coords: np.ndarray  # float64 [n_nodes, dim]
    cells: np.ndarray   # int32 [n_cells, nen]

    @property
    def dim(self) -> int:
        return ELEM_DIM[self.elem]

    @property
    def nen(self) -> int:
        return ELEM_NEN[self.elem]

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    @property
    def ndof(self) -> int:
        return self.dim * self.n_nodes


# ---------------------------------------------------------------- meshes

def quad_grid(nx: int, ny: int, h: float = 1.0) -> Mesh:
    """Structured nx x ny grid of h x h Q1 quads on [0, nx h] x [0, ny h]."""
    i, j = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
    coords = np.stack([i.ravel() * h, j.ravel() * h], axis=1).astype(np.float64)
    ei, ej = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ei, ej = ei.ravel(), ej.ravel()

    def nid(a, b):
        return a * (ny + 1) + b

    cells = np.stack([nid(ei, ej), nid(ei + 1, ej), nid(ei + 1, ej + 1), nid(ei, ej + 1)], axis=1)
    return Mesh(QUAD4, coords, cells.astype(np.int32))


def hex_grid(nx: int, ny: int, nz: int, h: float = 1.0) -> Mesh:
    """Structured nx x ny x nz grid of h-cubes (Q1 hexahedra)."""
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    coords = np.stack([i.ravel() * h, j.ravel() * h, k.ravel() * h], axis=1).astype(np.float64)
    ei, ej, ek = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ei, ej, ek = ei.ravel(), ej.ravel(), ek.ravel()

    def nid(a, b, c):
        return (a * (ny + 1) + b) * (nz + 1) + c

    cells = np.stack([
        nid(ei, ej, ek), nid(ei + 1, ej, ek), nid(ei + 1, ej + 1, ek), nid(ei, ej + 1, ek),
        nid(ei, ej, ek + 1), nid(ei + 1, ej, ek + 1), nid(ei + 1, ej + 1, ek + 1), nid(ei, ej + 1, ek + 1),
    ], axis=1)
    return Mesh(HEX8, coords, cells.astype(np.int32))


# Q2 hexahedron node order: the 8 corners as for Q1, then the other 19 points
# (a, b, c) / 2 of the 3 x 3 x 3 reference lattice, a, b, c in {0, 1, 2}, in
# ascending a + 3 b + 9 c.
_HEX27_LATTICE = [(0, 0, 0), (2, 0, 0), (2, 2, 0), (0, 2, 0), (0, 0, 2), (2, 0, 2), (2, 2, 2), (0, 2, 2)] + [
    (a, b, c) for c in range(3) for b in range(3) for a in range(3) if 1 in (a, b, c)]


def hex27_grid(nx: int, ny: int, nz: int, h: float = 1.0) -> Mesh:
    """Structured nx x ny x nz grid of h-cubes as Q2 hexahedra (27 nodes each,
    on the (2nx+1) x (2ny+1) x (2nz+1) lattice of spacing h/2)."""
    mx, my, mz = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    i, j, k = np.meshgrid(np.arange(mx), np.arange(my), np.arange(mz), indexing="ij")
    coords = np.stack([i.ravel() * 0.5 * h, j.ravel() * 0.5 * h, k.ravel() * 0.5 * h], axis=1).astype(np.float64)
    ei, ej, ek = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ei, ej, ek = ei.ravel(), ej.ravel(), ek.ravel()
    cells = np.stack([((2 * ei + a) * my + 2 * ej + b) * mz + 2 * ek + c for a, b, c in _HEX27_LATTICE], axis=1)
    return Mesh(HEX27, coords, cells.astype(np.int32))


def tri_grid(nx: int, ny: int, h: float = 1.0, jitter: float = 0.0,
             rng: Optional[np.random.Generator] = None) -> Mesh:
    """Each h-square split into 2 P1 triangles; interior nodes jittered by U(-jitter h, jitter h)."""
    q = quad_grid(nx, ny, h)
    coords = q.coords.copy()
    if jitter > 0.0:
        assert rng is not None
        i, j = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="ij")
        interior = ((i > 0) & (i < nx) & (j > 0) & (j < ny)).ravel()
        d = rng.uniform(-jitter * h, jitter * h, size=coords.shape)
        coords[interior] += d[interior]
    c = q.cells
    # square (i,j): [(i,j),(i+1,j),(i+1,j+1)] and [(i,j),(i+1,j+1),(i,j+1)], both CCW
    t0 = np.stack([c[:, 0], c[:, 1], c[:, 2]], axis=1)
    t1 = np.stack([c[:, 0], c[:, 2], c[:, 3]], axis=1)
    cells = np.stack([t0, t1], axis=1).reshape(-1, 3)
    return Mesh(TRI3, coords, cells.astype(np.int32))


def jitter_interior(mesh: Mesh, amount: float, rng: np.random.Generator) -> Mesh:
    """The same mesh with every node off the bounding box moved by
    U(-amount, amount) per coordinate (unit grids: Q1 cells become general,
    non-affine quadrilaterals or hexahedra; boundary nodes, hence supports and
    loads, stay put)."""
    x = mesh.coords
    lo, hi = x.min(axis=0), x.max(axis=0)
    inner = np.all((x > lo + 1e-9) & (x < hi - 1e-9), axis=1)
    c = x.copy()
    d = rng.uniform(-amount, amount, size=c.shape)
    c[inner] += d[inner]
    return Mesh(mesh.elem, c, mesh.cells)


# Kuhn split: one tetrahedron per permutation of the axes, walking from (0,0,0)
# to (1,1,1) one unit step at a time.
_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def skew_mesh(mesh: Mesh, kind: str) -> Mesh:
    """Coordinate maps that keep every Q1 element affine.

    'global': x -> A x with one fixed well-conditioned A (all Jacobians full).
    'kink': the last coordinate sheared by 0.4 (x0 - x_mid)_+, x_mid a grid
    plane, so elements left of it keep diagonal Jacobians and those right of
    it do not (a mesh with both kinds of element groups).
    """
    x = mesh.coords.copy()
    d = x.shape[1]
    if kind == "global":
        A = np.array([[1.0, 0.3, 0.1], [-0.2, 1.0, 0.25], [0.15, -0.1, 1.0]])[:d, :d]
        x = x @ A.T
    elif kind == "kink":
        xs = np.unique(x[:, 0])
        xm = xs[len(xs) // 2]
        x[:, d - 1] += 0.4 * np.maximum(x[:, 0] - xm, 0.0)
    else:
        raise ValueError(kind)
    return Mesh(mesh.elem, x, mesh.cells)


def _perm_sign(p):
    s = 1
    p = list(p)
    for a in range(3):
        for b in range(a + 1, 3):
            if p[a] > p[b]:
                s = -s
    return s


def kuhn_p2_tets(nx: int, ny: int, nz: int, h: float = 1.0, jitter: float = 0.0,
                 rng: Optional[np.random.Generator] = None) -> Mesh:
    """Cubes split into 6 Kuhn tetrahedra with quadratic (P2, 10-node) elements.

    P2 nodes are the full half-grid: node (I,J,K), 0 <= I <= 2nx etc., with id
    ``(I*(2ny+1)+J)*(2nz+1)+K``.  Vertices are the even half-grid points.
    """
    NX, NY, NZ = 2 * nx + 1, 2 * ny + 1, 2 * nz + 1
    I, J, K = np.meshgrid(np.arange(NX), np.arange(NY), np.arange(NZ), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()

    def hid(a, b, c):
        return (a * NY + b) * NZ + c

    # vertex coordinates on the lattice, jittered in the interior
    vi, vj, vk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    vx = np.stack([vi.ravel() * h, vj.ravel() * h, vk.ravel() * h], axis=1).astype(np.float64)
    if jitter > 0.0:
        assert rng is not None
        interior = ((vi > 0) & (vi < nx) & (vj > 0) & (vj < ny) & (vk > 0) & (vk < nz)).ravel()
        d = rng.uniform(-jitter * h, jitter * h, size=vx.shape)
        vx[interior] += d[interior]

    def vid(a, b, c):
        return (a * (ny + 1) + b) * (nz + 1) + c

    # every half-grid point is the midpoint of one mesh edge (or a vertex):
    # endpoints floor(P/2) and floor(P/2) + (odd coordinate unit vectors)
    lo = (I // 2, J // 2, K // 2)
    hi = (lo[0] + (I & 1), lo[1] + (J & 1), lo[2] + (K & 1))
    coords = 0.5 * (vx[vid(*lo)] + vx[vid(*hi)])

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    tets = []
    for perm in _PERMS:
        # vertex path in half-grid units
        path = [np.zeros(3, dtype=np.int64)]
        for ax in perm:
            nxt = path[-1].copy()
            nxt[ax] += 2
            path.append(nxt)
        if _perm_sign(perm) < 0:
            path[1], path[2] = path[2], path[1]
        verts = path
        nodes = list(verts) + [(verts[a] + verts[b]) // 2 for a, b in _EDGES]
        ids = [hid(2 * ci + n[0], 2 * cj + n[1], 2 * ck + n[2]) for n in nodes]
        tets.append(np.stack(ids, axis=1))
    cells = np.stack(tets, axis=1).reshape(-1, 10)
    return Mesh(TET10, coords, cells.astype(np.int32))


# ------------------------------------------------ boundary conditions and loads

def _close(a, b, tol=1e-9):
    return np.abs(a - b) < tol


def mbb_bc(mesh: Mesh):
    """MBB half-beam (Appendix B): x fixed on x=xmin, y fixed at (xmax, ymin), f_y=-1 at (xmin, ymax)."""
    x, y = mesh.coords[:, 0], mesh.coords[:, 1]
    xmin, xmax, ymin, ymax = x.min(), x.max(), y.min(), y.max()
    mask = np.zeros(mesh.ndof, dtype=np.uint8)
    mask[2 * np.nonzero(_close(x, xmin))[0] + 0] = 1
    mask[2 * np.nonzero(_close(x, xmax) & _close(y, ymin))[0] + 1] = 1
    f = np.zeros(mesh.ndof, dtype=np.float64)
    f[2 * np.nonzero(_close(x, xmin) & _close(y, ymax))[0] + 1] = -1.0
    return mask, f


def cantilever2d_bc(mesh: Mesh, load: str = "bottom_right"):
    """2D cantilever (Appendix A): x=xmin clamped; f_y=-1 at (xmax, ymin) or mid right edge."""
    x, y = mesh.coords[:, 0], mesh.coords[:, 1]
    xmin, xmax, ymin, ymax = x.min(), x.max(), y.min(), y.max()
    mask = np.zeros(mesh.ndof, dtype=np.uint8)
    fixed = np.nonzero(_close(x, xmin))[0]
    mask[2 * fixed] = 1
    mask[2 * fixed + 1] = 1
    f = np.zeros(mesh.ndof, dtype=np.float64)
    if load == "bottom_right":
        yl = ymin
    elif load == "mid_right":
        yl = 0.5 * (ymin + ymax)
    else:
        raise ValueError(load)
    f[2 * np.nonzero(_close(x, xmax) & _close(y, yl))[0] + 1] = -1.0
    return mask, f


def clamp_x0_bc(mesh: Mesh, load_edge: bool = True):
    """3D: x=xmin face clamped; f_y=-1 at every node of the edge x=xmax, y=ymin (Appendix C)."""
    x, y = mesh.coords[:, 0], mesh.coords[:, 1]
    xmin, xmax, ymin = x.min(), x.max(), y.min()
    mask = np.zeros(mesh.ndof, dtype=np.uint8)
    fixed = np.nonzero(_close(x, xmin))[0]
    for c in range(3):
        mask[3 * fixed + c] = 1
    f = np.zeros(mesh.ndof, dtype=np.float64)
    if load_edge:
        f[3 * np.nonzero(_close(x, xmax) & _close(y, ymin))[0] + 1] = -1.0
    return mask, f


# --------------------------------------------------------------- workloads

@dataclasses.dataclass
class Problem:
    name: str
    mesh: Mesh
    rho: np.ndarray         # float64 [n_cells]
    mask: np.ndarray        # uint8 [ndof]
    f: np.ndarray           # float64 [ndof]
    u: Optional[np.ndarray]  # float64 [ndof] (None: to be solved)
    E0: float = 1.0
    Emin: float = 1e-9
    nu: float = 0.3
    p: float = 3.0
    plane_strain: int = 0


def synthetic_u(rng: np.random.Generator, mask: np.ndarray) -> np.ndarray:
    u = rng.standard_normal(mask.shape[0])
    u[mask != 0] = 0.0
    return u


def mbb_q1(nx: int = 60, ny: int = 20, seed: int = 1001) -> Problem:
    """2D MBB half-beam of unit Q1 quads, rho ~ U(0.01, 1); u left to be solved."""
    rng = np.random.default_rng(seed)
    mesh = quad_grid(nx, ny)
    rho = rng.uniform(0.01, 1.0, mesh.n_cells)
    mask, f = mbb_bc(mesh)
    return Problem(f"mbb_q1_{nx}x{ny}", mesh, rho, mask, f, None)


def cantilever_tri(nx: int = 600, ny: int = 200, seed: int = 1002) -> Problem:
    """2D cantilever of jittered P1 triangles, rho ~ U(0.001, 1), synthetic u."""
    rng = np.random.default_rng(seed)
    mesh = tri_grid(nx, ny, jitter=0.2, rng=rng)
    rho = rng.uniform(0.001, 1.0, mesh.n_cells)
    mask, f = cantilever2d_bc(mesh, load="mid_right")
    u = synthetic_u(rng, mask)
    return Problem(f"cantilever_tri_{nx}x{ny}", mesh, rho, mask, f, u)


def cantilever_hex(nx: int = 120, ny: int = 40, nz: int = 40, seed: int = 1003,
                   skew: Optional[str] = None) -> Problem:
    """3D cantilever of unit Q1 hexes, rho ~ Beta(2, 2), synthetic u.

    skew maps the coordinates after the supports are chosen (skew_mesh)."""
    rng = np.random.default_rng(seed)
    mesh = hex_grid(nx, ny, nz)
    rho = rng.beta(2.0, 2.0, mesh.n_cells)
    mask, f = clamp_x0_bc(mesh)
    u = synthetic_u(rng, mask)
    if skew:
        mesh = skew_mesh(mesh, skew)
    return Problem(f"cantilever_hex_{nx}x{ny}x{nz}" + (f"_{skew}" if skew else ""), mesh, rho, mask, f, u)


def cantilever_hex27(nx: int = 60, ny: int = 20, nz: int = 20, h: float = 2.0, jitter: float = 0.15,
                     seed: int = 1005) -> Problem:
    """3D cantilever of Q2 hexahedra: nx x ny x nz cubes of side h (the
    defaults cover the 120 x 40 x 40 box of the Q1 cantilever with the same
    node lattice), every node off the bounding box moved by U(-jitter, jitter)
    per coordinate (curved, non-affine elements), rho ~ Beta(2, 2), synthetic u."""
    rng = np.random.default_rng(seed)
    mesh = hex27_grid(nx, ny, nz, h)
    if jitter:
        mesh = jitter_interior(mesh, jitter, rng)
    rho = rng.beta(2.0, 2.0, mesh.n_cells)
    mask, f = clamp_x0_bc(mesh)
    u = synthetic_u(rng, mask)
    return Problem(f"cantilever_hex27_{nx}x{ny}x{nz}", mesh, rho, mask, f, u)


def box_p2(n: int = 48, seed: int = 1004) -> Problem:
    """3D box of jittered Kuhn P2 tetrahedra, rho ~ U(0.001, 1), synthetic u."""
    rng = np.random.default_rng(seed)
    mesh = kuhn_p2_tets(n, n, n, jitter=0.15, rng=rng)
    rho = rng.uniform(0.001, 1.0, mesh.n_cells)
    mask, f = clamp_x0_bc(mesh, load_edge=False)
    u = synthetic_u(rng, mask)
    return Problem(f"box_p2_{n}", mesh, rho, mask, f, u)


def renumber(pr: Problem, seed: int) -> Problem:
    """The same problem with its nodes and elements renumbered by a seeded
    permutation: node i becomes pn[i], element k of the result is element
    pe[k] of pr (the nodal arrays and rho follow).  The permutations are
    returned in the name-independent attributes node_perm and elem_perm."""
    m0 = pr.mesh
    rng = np.random.default_rng(seed)
    pn, pe = rng.permutation(m0.n_nodes), rng.permutation(m0.n_cells)
    coords = np.empty_like(m0.coords)
    coords[pn] = m0.coords

    def nodal(v):
        if v is None:
            return None
        w = np.empty_like(v)
        w.reshape(-1, m0.dim)[pn] = v.reshape(-1, m0.dim)
        return w
    out = Problem(pr.name + "_renumbered", Mesh(m0.elem, coords, pn[m0.cells[pe]].astype(np.int32)),
                  pr.rho[pe], nodal(pr.mask), nodal(pr.f), nodal(pr.u), pr.E0, pr.Emin, pr.nu, pr.p)
    out.node_perm, out.elem_perm = pn, pe
    return out


def serving_request(rid: int):
    """One serving request: 2D Q1 n^2 (n in 32..512) or 3D Q1 n^3 (n in 16..96), p in {3, 4}."""
    rng = np.random.default_rng(5000 + rid)
    sizes = [("quad", 32), ("quad", 64), ("quad", 128), ("quad", 256), ("quad", 512),
             ("hex", 16), ("hex", 32), ("hex", 48), ("hex", 64), ("hex", 96)]
    kind, n = sizes[int(rng.integers(0, len(sizes)))]
    p = float(rng.choice([3.0, 4.0]))
    return kind, n, p, rng


def small_problem(elem: int, seed: int = 7, jitter: bool = True, dims=None, skew: Optional[str] = None) -> Problem:
    """Tiny meshes for oracle pins and parity tests (several tiles, ragged sizes).

    skew ('global' or 'kink', Q1 only) maps the coordinates after the supports
    are chosen (skew_mesh)."""
    rng = np.random.default_rng(seed)
    if elem == QUAD4:
        nx, ny = dims or (7, 5)
        mesh = quad_grid(nx, ny)
        mask, f = mbb_bc(mesh)
    elif elem == TRI3:
        nx, ny = dims or (7, 5)
        mesh = tri_grid(nx, ny, jitter=0.2 if jitter else 0.0, rng=rng)
        mask, f = cantilever2d_bc(mesh, load="mid_right")
    elif elem == HEX8:
        nx, ny, nz = dims or (5, 3, 4)
        mesh = hex_grid(nx, ny, nz)
        mask, f = clamp_x0_bc(mesh)
    elif elem == TET10:
        nx, ny, nz = dims or (3, 2, 2)
        mesh = kuhn_p2_tets(nx, ny, nz, jitter=0.15 if jitter else 0.0, rng=rng)
        mask, f = clamp_x0_bc(mesh)
    else:
        raise ValueError(elem)
    rho = rng.uniform(0.001, 1.0, mesh.n_cells)
    u = synthetic_u(rng, mask)
    if skew:
        if elem not in (QUAD4, HEX8):
            raise ValueError("skew applies to Q1 meshes")
        mesh = skew_mesh(mesh, skew)
    return Problem(f"small_{ELEM_NAMES[elem]}" + (f"_{skew}" if skew else ""), mesh, rho, mask, f, u)
