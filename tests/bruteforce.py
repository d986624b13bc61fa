"""Brute-force checkers for the oracle (tiny meshes only).

Nothing here calls the oracle's numbering or element code: the extruded mesh
is built as a plain 3D mesh (vertex (v, l) -> l*N0 + v, layer-major), every 3D
entity is found from the prisms as a set of 3D vertices, classified into the
entity types of Section 3.1.2 from its own vertices, and numbered by sorting.
Element integrals are computed in exact rational arithmetic from the
barycentric monomial formula, with no quadrature.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product
from math import factorial

import numpy as np


# ---------------------------------------------------------------------------
# Explicit 3D extruded mesh

def prism_entities(mesh, n_layers, layers=None):
    """Every prism's closure as sets of 3D vertex ids, in the stencil order
    (vertex 0, 1, 2; edge 0, 1, 2 opposite the vertex; cell), each closure
    entity split into (bottom horizontal, top horizontal, vertical) parts.
    layers: optional [N2, 2] range of layers present in each cell column."""
    n0 = mesh.n_vertices
    out = {}
    for c in range(mesh.n_cells):
        v = [int(x) for x in mesh.cell_vertex[c]]
        l_lo, l_hi = (0, n_layers) if layers is None else (int(layers[c][0]), int(layers[c][1]))
        for l in range(l_lo, l_hi):
            bot = [x + l * n0 for x in v]
            top = [x + (l + 1) * n0 for x in v]
            closure = []
            for a in range(3):
                closure.append((frozenset([bot[a]]), frozenset([top[a]]), frozenset([bot[a], top[a]])))
            for a in range(3):
                p, q = (a + 1) % 3, (a + 2) % 3
                closure.append((frozenset([bot[p], bot[q]]), frozenset([top[p], top[q]]),
                                frozenset([bot[p], bot[q], top[p], top[q]])))
            closure.append((frozenset(bot), frozenset(top), frozenset(bot + top)))
            out[(c, l)] = closure
    return out


def classify(ent: frozenset, mesh, edge_index, cell_index):
    """Entity type (d1, d2), base entity index i and level l of a 3D entity."""
    n0 = mesh.n_vertices
    base = sorted({x % n0 for x in ent})
    levels = sorted({x // n0 for x in ent})
    d1 = len(base) - 1
    d2 = len(levels) - 1
    if d1 == 0:
        i = base[0]
    elif d1 == 1:
        i = edge_index[tuple(base)]
    else:
        i = cell_index[frozenset(base)]
    return (d1, d2), i, levels[0]


def bruteforce_numbering(mesh, n_layers, delta, layers=None, dofs=None):
    """Vertical-innermost numbering obtained by sorting all (entity, j) keys
    of the explicit 3D mesh by (d1, i, l, d2, j).

    dofs: optional per-entity counts, dofs[d1][i] = (horizontal, vertical),
    in place of the per-type table delta.

    Returns (numbers, stencils): numbers[((d1, d2), i, l)] = first DoF,
    stencils[(c, l)] = the DoF list of that prism in stencil order."""
    delta = np.asarray(delta).reshape(3, 2)

    def count(d1, i, d2):
        return int(dofs[d1][i][d2]) if dofs is not None else int(delta[d1, d2])

    edge_index = {(int(a), int(b)): e for e, (a, b) in enumerate(mesh.edge_vertex)}
    cell_index = {frozenset(int(x) for x in mesh.cell_vertex[c]): c for c in range(mesh.n_cells)}
    prisms = prism_entities(mesh, n_layers, layers)
    entities = {}
    for closure in prisms.values():
        for parts in closure:
            for ent in parts:
                if ent not in entities:
                    entities[ent] = classify(ent, mesh, edge_index, cell_index)
    keys = []
    for ent, ((d1, d2), i, l) in entities.items():
        for j in range(count(d1, i, d2)):
            keys.append((d1, i, l, d2, j))
    keys.sort()
    first = {}
    for n, (d1, i, l, d2, j) in enumerate(keys):
        if j == 0:
            first[((d1, d2), i, l)] = n
    stencils = {}
    for (c, l), closure in prisms.items():
        row = []
        for bot, top, vert in closure:
            (d1, _), ib, lb = entities[bot]
            nh = count(d1, ib, 0)
            nv = count(d1, ib, 1)
            row += [first[((d1, 0), ib, lb)] + j for j in range(nh)]
            (_, _), it, lt = entities[top]
            row += [first[((d1, 0), it, lt)] + j for j in range(nh)]
            (_, _), iv, lv = entities[vert]
            row += [first[((d1, 1), iv, lv)] + j for j in range(nv)]
        stencils[(c, l)] = row
    return len(keys), first, stencils, entities


# ---------------------------------------------------------------------------
# Exact element integrals on the reference prism (barycentric monomials)

def _tri_monomial(i, j, k):
    """Integral of l0^i l1^j l2^k over the reference triangle (area 1/2)."""
    return Fraction(factorial(i) * factorial(j) * factorial(k), factorial(i + j + k + 2))


def _pmul(a, b):
    out = {}
    for ka, va in a.items():
        for kb, vb in b.items():
            k = tuple(x + y for x, y in zip(ka, kb))
            out[k] = out.get(k, 0) + va * vb
    return out


def _vmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


E = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]


def h_poly(h, d, ent, alpha):
    """Horizontal basis functions as barycentric polynomials {exponents: coeff}."""
    if h == "CG1":
        return {E[ent]: Fraction(1)}
    if h == "CG2":
        if d == 0:
            sq = tuple(2 * x for x in E[ent])
            return {sq: Fraction(2), E[ent]: Fraction(-1)}
        a, b = (ent + 1) % 3, (ent + 2) % 3
        return {tuple(x + y for x, y in zip(E[a], E[b])): Fraction(4)}
    if h == "DG0":
        return {(0, 0, 0): Fraction(1)}
    if h == "DG1":
        return {E[alpha]: Fraction(1)}
    raise ValueError(h)


def v_poly(v, part, beta):
    """Vertical basis functions as coefficient lists in zeta."""
    F = Fraction
    if part == "bot":
        return [F(1), F(-1)] if v == "CG1" else [F(1), F(-3), F(2)]
    if part == "top":
        return [F(0), F(1)] if v == "CG1" else [F(0), F(-1), F(2)]
    if v == "CG2":
        return [F(0), F(4), F(-4)]
    if v == "DG0":
        return [F(1)]
    if v == "DG1":
        return [F(1), F(-1)] if beta == 0 else [F(0), F(1)]
    raise ValueError(v)


H_NODES = {"CG1": (1, 0, 0), "CG2": (1, 1, 0), "DG0": (0, 0, 1), "DG1": (0, 0, 3)}
V_NODES = {"CG1": (1, 0), "CG2": (1, 1), "DG0": (0, 1), "DG1": (0, 2)}


def local_basis(h, v):
    """[(horizontal poly, vertical poly)] per stencil position."""
    out = []
    for e in range(7):
        d = 0 if e < 3 else (1 if e < 6 else 2)
        ent = e if d == 0 else (e - 3 if d == 1 else 0)
        nh = H_NODES[h][d] * V_NODES[v][0]
        nv = H_NODES[h][d] * V_NODES[v][1]
        for part, count, nvp in (("bot", nh, V_NODES[v][0]), ("top", nh, V_NODES[v][0]), ("int", nv, V_NODES[v][1])):
            for j in range(count):
                alpha, beta = divmod(j, nvp)
                out.append((h_poly(h, d, ent, alpha), v_poly(v, part, beta)))
    return out


def _integrate(hp, vp):
    th = sum((c * _tri_monomial(*k) for k, c in hp.items()), Fraction(0))
    tv = sum((c / (n + 1) for n, c in enumerate(vp)), Fraction(0))
    return th * tv


def reference_tensors(h, v, order):
    """R[c][idx] = integral over the reference prism of the product of `order`
    basis functions (indices idx) times lambda_c, for c = 0, 1, 2."""
    basis = local_basis(h, v)
    k = len(basis)
    R = []
    for c in range(3):
        lam_c = {E[c]: Fraction(1)}
        T = {}
        for idx in product(range(k), repeat=order):
            if tuple(sorted(idx)) != idx:
                continue
            hp = lam_c
            vp = [Fraction(1)]
            for p in idx:
                hp = _pmul(hp, basis[p][0])
                vp = _vmul(vp, basis[p][1])
            T[idx] = _integrate(hp, vp)
        R.append(T)
    return R, k


def prism_geometry(mesh_xy, vcoords, cell_vertex, c, l):
    """Exact |twice the triangle area| and the three column heights of prism (c, l)."""
    v = [int(x) for x in cell_vertex[c]]
    P = [[Fraction(float(mesh_xy[a, 0])), Fraction(float(mesh_xy[a, 1]))] for a in v]
    twoA = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[2][0] - P[0][0]) * (P[1][1] - P[0][1])
    hts = [Fraction(float(vcoords[a, l + 1, 2])) - Fraction(float(vcoords[a, l, 2])) for a in v]
    return abs(twoA), hts


def _lookup(T, idx):
    return T[tuple(sorted(idx))]


def exact_mass(mesh, vcoords, n_layers, space, stencils, n_dofs, f):
    """b_i = integral of f_h v_i, exactly, for f given at the DoFs."""
    h, v = space
    R, k = reference_tensors(h, v, 2)
    fq = [Fraction(float(x)) for x in f]
    b = [Fraction(0)] * n_dofs
    for (c, l), row in stencils.items():
        twoA, hts = prism_geometry(mesh.xy, vcoords, mesh.cell_vertex, c, l)
        for p in range(k):
            s = Fraction(0)
            for q in range(k):
                m = sum(hts[cc] * _lookup(R[cc], (p, q)) for cc in range(3))
                s += m * fq[row[q]]
            b[row[p]] += twoA * s
    return b


def exact_cubic(mesh, vcoords, n_layers, stencils, n_dofs, u, f):
    """F_i = integral of (u_h^3 - f_h) v_i exactly, P1 x P1."""
    R2, k = reference_tensors("CG1", "CG1", 2)
    R4, _ = reference_tensors("CG1", "CG1", 4)
    uq = [Fraction(float(x)) for x in u]
    fq = [Fraction(float(x)) for x in f]
    F = [Fraction(0)] * n_dofs
    for (c, l), row in stencils.items():
        twoA, hts = prism_geometry(mesh.xy, vcoords, mesh.cell_vertex, c, l)
        ul = [uq[r] for r in row]
        fl = [fq[r] for r in row]
        for p in range(k):
            s = Fraction(0)
            for cc in range(3):
                acc = Fraction(0)
                for q in range(k):
                    for r in range(k):
                        for t in range(k):
                            acc += _lookup(R4[cc], (p, q, r, t)) * ul[q] * ul[r] * ul[t]
                for q in range(k):
                    acc -= _lookup(R2[cc], (p, q)) * fl[q]
                s += hts[cc] * acc
            F[row[p]] += twoA * s
    return F


def exact_cubic_vjp(mesh, vcoords, n_layers, stencils, n_dofs, u, w):
    """g_i = integral of 3 u_h^2 w_h v_i exactly, P1 x P1 (the derivative of
    the cubic residual's u^3 term applied to w)."""
    R4, k = reference_tensors("CG1", "CG1", 4)
    uq = [Fraction(float(x)) for x in u]
    wq = [Fraction(float(x)) for x in w]
    g = [Fraction(0)] * n_dofs
    for (c, l), row in stencils.items():
        twoA, hts = prism_geometry(mesh.xy, vcoords, mesh.cell_vertex, c, l)
        ul = [uq[r] for r in row]
        wl = [wq[r] for r in row]
        for p in range(k):
            s = Fraction(0)
            for cc in range(3):
                acc = Fraction(0)
                for q in range(k):
                    for r in range(k):
                        for t in range(k):
                            acc += _lookup(R4[cc], (p, q, r, t)) * ul[q] * ul[r] * wl[t]
                s += hts[cc] * 3 * acc
            g[row[p]] += twoA * s
    return g
