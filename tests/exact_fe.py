"""Exact rational finite-element integrals for pinning the oracle (tests only).

An independent route to K_e^0: the isotropic bilinear form
    a(u, v) = int lambda div(u) div(v) + 2 mu eps(u):eps(v) dx
(plane stress: lambda replaced by lambda* = E nu / (1 - nu^2)), with basis
functions written as sympy polynomials on the reference element, mapped by
an affine map with rational vertices and integrated exactly by the monomial
formulas
    unit cube:     int x^a y^b z^c = 1 / ((a+1)(b+1)(c+1))
    unit simplex:  int x^a y^b z^c = a! b! c! / (a+b+c+d)!   (d = dimension).
Nothing here shares code with the oracle (which uses the Voigt D matrix, the
B matrix and numerical quadrature).
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial

import sympy as sp

X = sp.symbols("x0:3")


def _lagrange_1d(k, t):
    """Quadratic Lagrange polynomial of node k of {0, 1/2, 1}, by the product
    formula prod_{m != k} (t - t_m) / (t_k - t_m)."""
    nodes = [sp.Integer(0), sp.Rational(1, 2), sp.Integer(1)]
    p = sp.Integer(1)
    for m in range(3):
        if m != k:
            p *= (t - nodes[m]) / (nodes[k] - nodes[m])
    return sp.expand(p)


# Q2 hexahedron: corners as for Q1 (lattice 0/2), then the other lattice
# points in ascending a + 3b + 9c
HEX27_LATTICE = [(0, 0, 0), (2, 0, 0), (2, 2, 0), (0, 2, 0), (0, 0, 2), (2, 0, 2), (2, 2, 2), (0, 2, 2)] + [
    (a, b, c) for c in range(3) for b in range(3) for a in range(3) if a == 1 or b == 1 or c == 1]


def _ref_basis(elem):
    x, y, z = X
    if elem == 5:  # Q2 hex on [0,1]^3
        return [sp.expand(_lagrange_1d(a, x) * _lagrange_1d(b, y) * _lagrange_1d(c, z))
                for a, b, c in HEX27_LATTICE], 3, "cube"
    if elem == 1:  # Q1 quad on [0,1]^2, CCW from the origin
        c = [(0, 0), (1, 0), (1, 1), (0, 1)]
        f = lambda b, t: t if b else 1 - t
        return [sp.expand(f(a, x) * f(b, y)) for a, b in c], 2, "cube"
    if elem == 3:  # Q1 hex on [0,1]^3, bottom then top face CCW
        c = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
        f = lambda b, t: t if b else 1 - t
        return [sp.expand(f(a, x) * f(b, y) * f(cc, z)) for a, b, cc in c], 3, "cube"
    if elem == 2:  # P1 triangle
        return [1 - x - y, x, y], 2, "simplex"
    if elem == 4:  # P2 tetrahedron
        L = [1 - x - y - z, x, y, z]
        edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
        phis = [sp.expand(L[i] * (2 * L[i] - 1)) for i in range(4)]
        phis += [sp.expand(4 * L[a] * L[b]) for a, b in edges]
        return phis, 3, "simplex"
    raise ValueError(elem)


def _integrate_ref(poly, dim, kind):
    P = sp.Poly(poly, *X[:dim])
    total = sp.Rational(0)
    for monom, coeff in P.terms():
        if kind == "cube":
            v = sp.Rational(1)
            for a in monom:
                v /= (a + 1)
        else:
            num = 1
            for a in monom:
                num *= factorial(a)
            v = sp.Rational(num, factorial(sum(monom) + dim))
        total += coeff * v
    return total


def exact_ke0(elem, verts, nu=Fraction(3, 10), plane_strain=False):
    """Exact K_e^0 (E = 1) for an affine element.

    verts: the dim+1 (simplex) or corner (Q1: nodes 0, 1 / 0, 1, 3 / 0, 1, 3, 4)
    rational vertex coordinates that define the affine map x = x0 + J xi.
    Returns a sympy Matrix of rationals, dof order interleaved (node, comp).
    """
    phis, dim, kind = _ref_basis(elem)
    nu = sp.Rational(nu)
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1 / (2 * (1 + nu))
    if dim == 2 and not plane_strain:
        lam = 2 * lam * mu / (lam + 2 * mu)
    # affine map columns
    if elem == 1:
        cols = [1, 3]
    elif elem in (3, 5):
        cols = [1, 3, 4]
    else:
        cols = list(range(1, dim + 1))
    x0 = [sp.Rational(v) for v in verts[0]]
    J = sp.Matrix(dim, dim, lambda a, m: sp.Rational(verts[cols[m]][a]) - x0[a])
    detJ = J.det()
    G = J.inv()  # G[m, a] = d xi_m / d x_a
    grads = []
    for ph in phis:
        gref = [sp.diff(ph, X[m]) for m in range(dim)]
        grads.append([sp.expand(sum(gref[m] * G[m, a] for m in range(dim))) for a in range(dim)])
    nen = len(phis)
    ldof = dim * nen
    K = sp.zeros(ldof, ldof)
    for i in range(nen):
        for j in range(nen):
            for a in range(dim):
                for b in range(dim):
                    # a(phi_j e_b, phi_i e_a)
                    integrand = lam * grads[i][a] * grads[j][b] + mu * grads[i][b] * grads[j][a]
                    if a == b:
                        integrand += mu * sum(grads[i][k] * grads[j][k] for k in range(dim))
                    K[dim * i + a, dim * j + b] = abs(detJ) * _integrate_ref(sp.expand(integrand), dim, kind)
    return K


def exact_ref_moments(elem):
    """M[i][j][m][n] = int_ref d_m phi_i d_n phi_j (exact rationals)."""
    phis, dim, kind = _ref_basis(elem)
    nen = len(phis)
    g = [[sp.diff(ph, X[m]) for m in range(dim)] for ph in phis]
    return [[[[_integrate_ref(sp.expand(g[i][m] * g[j][n]), dim, kind) for n in range(dim)]
              for m in range(dim)] for j in range(nen)] for i in range(nen)]


def exact_energy(elem, verts, U, nu=Fraction(3, 10)):
    """a(u, u) exactly for the field u = sum_i U[i] phi_i of an affine 3D
    element (E = 1), U rational nodal values [nen][3]: the same affine map as
    exact_ke0, integrand lambda div(u)^2 + 2 mu eps(u):eps(u)."""
    phis, dim, kind = _ref_basis(elem)
    nu = sp.Rational(nu)
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1 / (2 * (1 + nu))
    cols = [1, 3, 4] if elem in (3, 5) else list(range(1, dim + 1))
    x0 = [sp.Rational(v) for v in verts[0]]
    J = sp.Matrix(dim, dim, lambda a, m: sp.Rational(verts[cols[m]][a]) - x0[a])
    G = J.inv()
    uref = [sp.expand(sum(sp.Rational(U[i][a]) * phis[i] for i in range(len(phis)))) for a in range(dim)]
    grad = [[sp.expand(sum(sp.diff(uref[a], X[m]) * G[m, b] for m in range(dim))) for b in range(dim)]
            for a in range(dim)]
    div = sum(grad[a][a] for a in range(dim))
    ee = sum(((grad[a][b] + grad[b][a]) / 2) ** 2 for a in range(dim) for b in range(dim))
    return abs(J.det()) * _integrate_ref(sp.expand(lam * div ** 2 + 2 * mu * ee), dim, kind)
