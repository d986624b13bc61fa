"""CPU oracle for the extruded-mesh numbering and column iteration.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
It shares no code with the HIP path; the only common module is the seeded
input generator.

Reference: Bercea et al., arXiv 1604.05937.
* Algorithm 1 (Section 3.2) -- vertical-innermost numbering, in ``number``
  (a literal counter loop in ``oracle.c``).
* Algorithm 2 (Section 3.3) -- vertical offsets, in ``stencil``.
* Algorithm 3 (Section 3.3) -- column iteration ``L + n * offset`` with a
  stencil kernel, in ``par_loop``.
* The kernels integrate the forms of Section 4.1.1 (the residual of the
  integral of f v) and the mass action, cubic residual and its derivatives,
  by quadrature with a full Jacobian at each point.  The rules are Gauss
  rules from scipy (Gauss-Legendre on the interval; the collapsed
  Gauss-Jacobi conical product on the triangle), chosen exact for the
  polynomial degree each form reaches on a prism whose columns are vertical
  (x, y fixed along a column, any z).

Readings where the paper is silent (each also listed in the design notes):
* entities are visited dimension-major (d1 = 0, 1, 2), then by base index;
* several DoFs on one entity are ordered horizontal-node major, vertical-node
  minor;
* a prism's stencil lists its closure entities as vertex 0, 1, 2, edge 0, 1,
  2 (edge a opposite vertex a), cell; per entity the bottom horizontal DoFs,
  the top horizontal DoFs, then the vertical DoFs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from functools import lru_cache

import numpy as np
from scipy.special import roots_jacobi, roots_legendre

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FORM_MASS = 1
FORM_CUBIC = 2
FORM_CUBIC_VJP = 3
FORM_CUBIC_JVP = 4
FORM_CUBIC_FUSED = 5
FORM_MASS_ABS = 6
FORM_CUBIC_ABS = 7
FORM_VJP_ABS = 8

# bilinear forms assembled into a matrix (oracle_assemble)
ASM_MASS = 1          # integral phi_j phi_i
ASM_CUBIC_JAC = 2     # integral 3 u^2 phi_j phi_i, the Jacobian of integral (u^3 - f) v
ASM_MASS_ABS = 3
ASM_CUBIC_JAC_ABS = 4


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                        _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


@lru_cache(maxsize=1)
def _lib():
    # ORACLE_LIB names another build of oracle.c (the sanitizer build of the
    # tests); by default the plain build next to the source
    path = os.environ.get("ORACLE_LIB", "")
    if not path:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        path = _LIB
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.oracle_alg1_number.restype = ctypes.c_int64
    lib.oracle_alg1_number.argtypes = [P, ctypes.c_int32, P, P, P, P]
    lib.oracle_stencil.restype = ctypes.c_int32
    lib.oracle_stencil.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P, P, P, P]
    lib.oracle_alg1_number_var.restype = ctypes.c_int64
    lib.oracle_alg1_number_var.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P, P, P, P, P]
    lib.oracle_stencil_var.restype = ctypes.c_int32
    lib.oracle_stencil_var.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P, P, P]
    lib.oracle_par_loop.restype = None
    lib.oracle_par_loop.argtypes = [ctypes.c_int32, ctypes.c_int64, P, ctypes.c_int32, P,
                                    P, P, P, ctypes.c_int32, P, P,
                                    P, P, P, P, P, P, ctypes.c_int32,
                                    ctypes.c_int32, P, P, P, P]
    lib.oracle_alg1_number_mixed.restype = ctypes.c_int64
    lib.oracle_alg1_number_mixed.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P]
    lib.oracle_stencil_mixed.restype = ctypes.c_int64
    lib.oracle_stencil_mixed.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, P, P, P, P, P, P, P, P, P]
    lib.oracle_facet_loop.restype = None
    lib.oracle_facet_loop.argtypes = [ctypes.c_int64, P, ctypes.c_int32, P, P, P, ctypes.c_int32, P, P, P, P,
                                      ctypes.c_int32, ctypes.c_int32, P, P, P, P, P]
    lib.oracle_greedy_colour.restype = ctypes.c_int32
    lib.oracle_greedy_colour.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P]
    lib.oracle_assemble.restype = None
    lib.oracle_assemble.argtypes = [ctypes.c_int32, ctypes.c_int64, P, ctypes.c_int32, P, P, P,
                                    ctypes.c_int32, P, P, P, P, P, P,
                                    ctypes.c_int32, P, P, P, P]
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Finite element families on the prism (tensor products, Section 3.1.1 and
# Section 4.1.2).  Horizontal families live on the triangle, vertical ones on
# the interval; a space is a pair (h, v).

# number of horizontal nodes carried by a base entity of dimension 0, 1, 2
_H_NODES = {"CG1": (1, 0, 0), "CG2": (1, 1, 0), "DG0": (0, 0, 1), "DG1": (0, 0, 3)}
# number of vertical nodes on an interval end point and in its interior
_V_NODES = {"CG1": (1, 0), "CG2": (1, 1), "DG0": (0, 1), "DG1": (0, 2)}


def delta_table(h: str, v: str) -> np.ndarray:
    """delta((d1, d2)) for the tensor-product space h x v, as a [3, 2] table."""
    hn = _H_NODES[h]
    vn = _V_NODES[v]
    return np.array([[hn[d] * vn[0], hn[d] * vn[1]] for d in range(3)], dtype=np.int32)


def _h_basis(h: str, d: int, ent: int, j: int, lam):
    """Horizontal basis function of node j on closure entity ``ent`` (local
    index within its dimension) evaluated at barycentric coordinates lam[3]."""
    if h == "CG1":
        return lam[ent]
    if h == "CG2":
        if d == 0:
            return lam[ent] * (2.0 * lam[ent] - 1.0)
        a, b = (ent + 1) % 3, (ent + 2) % 3
        return 4.0 * lam[a] * lam[b]
    if h == "DG0":
        return np.ones_like(lam[0])
    if h == "DG1":
        return lam[j]
    raise ValueError(h)


def _v_basis(v: str, part: str, j: int, z):
    """Vertical basis function: part 'bot' / 'top' endpoint node or interior node j."""
    if part == "bot":
        return (1.0 - z) if v == "CG1" else (1.0 - z) * (1.0 - 2.0 * z)
    if part == "top":
        return z if v == "CG1" else z * (2.0 * z - 1.0)
    if v == "CG2":
        return 4.0 * z * (1.0 - z)
    if v == "DG0":
        return np.ones_like(z)
    if v == "DG1":
        return (1.0 - z) if j == 0 else z
    raise ValueError(v)


def stencil_layout(h: str, v: str):
    """For each stencil position p: (entity dim d, local entity, part, horizontal
    node index alpha within the entity, vertical node index beta)."""
    dl = delta_table(h, v)
    hn = _H_NODES[h]
    vn = _V_NODES[v]
    out = []
    for e in range(7):
        d = 0 if e < 3 else (1 if e < 6 else 2)
        ent = e if d == 0 else (e - 3 if d == 1 else 0)
        for part, count, nvp in (("bot", dl[d, 0], vn[0]), ("top", dl[d, 0], vn[0]), ("int", dl[d, 1], vn[1])):
            for j in range(count):
                alpha, beta = divmod(j, nvp) if nvp else (j, 0)
                out.append((d, ent, part, alpha, beta))
    assert len(out) == sum(2 * dl[d, 0] + dl[d, 1] for d in (0, 0, 0, 1, 1, 1, 2))
    del hn
    return out


def tabulate(h: str, v: str, pts: np.ndarray) -> np.ndarray:
    """phi[q, p] for the space h x v at reference points pts[q] = (xi, eta, zeta)."""
    lam = np.stack([1.0 - pts[:, 0] - pts[:, 1], pts[:, 0], pts[:, 1]])
    z = pts[:, 2]
    cols = []
    for d, ent, part, alpha, beta in stencil_layout(h, v):
        cols.append(_h_basis(h, d, ent, alpha, lam) * _v_basis(v, part, beta, z))
    return np.stack(cols, axis=1)


def tabulate_coords(pts: np.ndarray):
    """P1 x P1 basis of the coordinate field and its reference derivatives."""
    phi = tabulate("CG1", "CG1", pts)
    nq = pts.shape[0]
    dphi = np.zeros((nq, 6, 3))
    dlam = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])  # d lambda_a / d(xi, eta)
    lam = np.stack([1.0 - pts[:, 0] - pts[:, 1], pts[:, 0], pts[:, 1]], axis=1)
    z = pts[:, 2]
    for a in range(3):
        for beta, (vz, dvz) in enumerate(((1.0 - z, -1.0), (z, 1.0))):
            p = 2 * a + beta
            dphi[:, p, 0] = dlam[a, 0] * vz
            dphi[:, p, 1] = dlam[a, 1] * vz
            dphi[:, p, 2] = lam[:, a] * dvz
    return phi, dphi


# ---------------------------------------------------------------------------
# Quadrature

def gauss_legendre01(m: int):
    """m-point Gauss-Legendre rule on [0, 1] (exact to degree 2m-1)."""
    x, w = roots_legendre(m)
    return 0.5 * (x + 1.0), 0.5 * w


def triangle_rule(n: int):
    """Conical-product rule on the reference triangle {xi, eta >= 0, xi+eta <= 1}
    with n*n points, exact to total degree 2n-1: xi = u, eta = t (1 - u), with u
    from n-point Gauss-Jacobi (weight 1-u) and t from n-point Gauss-Legendre."""
    xj, wj = roots_jacobi(n, 1.0, 0.0)
    u = 0.5 * (xj + 1.0)
    wu = 0.25 * wj
    t, wt = gauss_legendre01(n)
    pts = np.array([[ui, ti * (1.0 - ui)] for ui in u for ti in t])
    wts = np.array([a * b for a in wu for b in wt])
    return pts, wts


def prism_rule(n_tri: int, n_int: int):
    tp, tw = triangle_rule(n_tri)
    zp, zw = gauss_legendre01(n_int)
    pts = np.array([[p[0], p[1], z] for p in tp for z in zp])
    wts = np.array([a * b for a in tw for b in zw])
    return pts, wts


# Highest polynomial degree (horizontal, vertical) of each form's integrand on
# vertical-column prisms: det J is linear in the horizontal variables there.
_DEG_V = {"CG1": 1, "CG2": 2, "DG0": 0, "DG1": 1}
_DEG_H = {"CG1": 1, "CG2": 2, "DG0": 0, "DG1": 1}


def rule_for(form: int, h: str, v: str):
    dh, dv = _DEG_H[h], _DEG_V[v]
    if form in (FORM_MASS, FORM_MASS_ABS):
        nh, nv = 2 * dh + 1, 2 * dv
    else:  # cubic family: four field factors times a test function
        nh, nv = 4 * dh + 1, 4 * dv
    n_tri = max(1, (nh + 2) // 2)
    n_int = max(1, (nv + 2) // 2)
    return prism_rule(n_tri, n_int)


# ---------------------------------------------------------------------------
# Numbering

@dataclass
class Numbering:
    counts: tuple
    n_layers: int
    delta: np.ndarray           # [3, 2]
    n_dofs: int
    first: list                 # first[d1]: [N_d1, lam+1, 2] int64 (-1 = no entity)
    lmap: np.ndarray            # [N2, k] int64 explicit list at the column's bottom layer
    offsets: np.ndarray         # [k] int32
    entity_dim: np.ndarray      # [k] int32
    lo: list = None             # variable layers: first layer of every entity column, per dimension
    hi: list = None             # ... and one past its last layer
    cell_lam: np.ndarray = None  # variable layers: layers of every cell column (int32)

    @property
    def k(self) -> int:
        return int(self.offsets.size)

    def column_starts(self, d1: int) -> np.ndarray:
        """First DoF of the column of every base entity of dimension d1."""
        if self.lo is None:
            return self.first[d1][:, 0, 0].copy()
        idx = np.arange(self.first[d1].shape[0])
        return self.first[d1][idx, self.lo[d1], 0].copy()


def entity_layers(counts, n_layers: int, cell_vertex, cell_edge, layers):
    """Layer ranges of every entity column when each cell c carries the prisms
    of layers[c, 0] .. layers[c, 1] - 1 (reading: a vertex or edge column spans
    the union of the ranges of the cells around it)."""
    layers = np.asarray(layers, dtype=np.int32).reshape(-1, 2)
    n0, n1, n2 = (int(x) for x in counts)
    assert layers.shape[0] == n2
    assert np.all(layers[:, 0] >= 0) and np.all(layers[:, 0] < layers[:, 1]) and np.all(layers[:, 1] <= n_layers)
    lo = [np.full(n0, n_layers, np.int32), np.full(n1, n_layers, np.int32), layers[:, 0].copy()]
    hi = [np.zeros(n0, np.int32), np.zeros(n1, np.int32), layers[:, 1].copy()]
    for c in range(n2):
        for a in range(3):
            v = cell_vertex[c, a]
            lo[0][v] = min(lo[0][v], layers[c, 0])
            hi[0][v] = max(hi[0][v], layers[c, 1])
            if cell_edge is not None:
                e = cell_edge[c, a]
                lo[1][e] = min(lo[1][e], layers[c, 0])
                hi[1][e] = max(hi[1][e], layers[c, 1])
    if cell_edge is None:
        lo[1][:] = 0
        hi[1][:] = n_layers
    return lo, hi


def number(counts, n_layers: int, delta, cell_vertex, cell_edge=None, layers=None) -> Numbering:
    """Algorithm 1 + the explicit lists + Algorithm 2 for one function space.

    layers: optional [N2, 2] layer range per cell (variable layers); n_layers
    is then the largest layer count."""
    lib = _lib()
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    delta = np.ascontiguousarray(np.asarray(delta, dtype=np.int32).reshape(3, 2))
    if n_layers < 1:
        raise ValueError("need at least one layer")
    # dimensions without DoFs get no table (the counter loop still visits them)
    first = [np.full((int(counts[d]), n_layers + 1, 2), -1, dtype=np.int64) if delta[d].sum() else None
             for d in range(3)]
    n_dofs = lib.oracle_alg1_number(_ptr(counts), n_layers, _ptr(delta), _ptr(first[0]), _ptr(first[1]), _ptr(first[2]))
    k = lib.oracle_stencil(0, n_layers, _ptr(delta), None, None, None, None, None, None, None, None)
    offsets = np.zeros(k, dtype=np.int32)
    edim = np.zeros(k, dtype=np.int32)
    lmap = np.zeros((int(counts[2]), k), dtype=np.int64)
    cv = np.ascontiguousarray(cell_vertex, dtype=np.int32)
    if delta[1].sum() > 0:
        if cell_edge is None:
            raise ValueError("this space has edge DoFs: cell_edge is required")
        ce = np.ascontiguousarray(cell_edge, dtype=np.int32)
    else:
        ce = None
    lib.oracle_stencil(int(counts[2]), n_layers, _ptr(delta), _ptr(cv), _ptr(ce),
                       _ptr(first[0]), _ptr(first[1]), _ptr(first[2]), _ptr(lmap), _ptr(offsets), _ptr(edim))
    if layers is None:
        return Numbering(tuple(int(x) for x in counts), n_layers, delta, int(n_dofs), first, lmap, offsets, edim)
    # variable layers: number again over every entity's own range
    lo, hi = entity_layers(counts, n_layers, np.asarray(cell_vertex), None if cell_edge is None else
                           np.asarray(cell_edge), layers)
    for d in range(3):
        if first[d] is not None:
            first[d][:] = -1
    n_dofs = lib.oracle_alg1_number_var(_ptr(counts), n_layers, _ptr(delta), _ptr(lo[0]), _ptr(hi[0]), _ptr(lo[1]),
                                        _ptr(hi[1]), _ptr(lo[2]), _ptr(hi[2]),
                                        _ptr(first[0]), _ptr(first[1]), _ptr(first[2]))
    cell_lo = np.ascontiguousarray(lo[2])
    lib.oracle_stencil_var(int(counts[2]), n_layers, _ptr(delta), _ptr(cv), _ptr(ce), _ptr(cell_lo),
                           _ptr(first[0]), _ptr(first[1]), _ptr(first[2]), _ptr(lmap))
    return Numbering(tuple(int(x) for x in counts), n_layers, delta, int(n_dofs), first, lmap, offsets, edim,
                     lo, hi, np.ascontiguousarray(hi[2] - lo[2], dtype=np.int32))


@dataclass
class MixedNumbering:
    """Algorithm 1 with a DoF count per entity: dofs[d1] is [N_d1, 2]
    (horizontal, vertical DoFs of every base entity of dimension d1)."""
    counts: tuple
    n_layers: int
    dofs: list
    n_dofs: int
    first: list                 # first[d1]: [N_d1, lam+1, 2] int64
    list_off: np.ndarray        # [N2 + 1] int64
    lmap: np.ndarray            # [list_off[-1]] int64, bottom-layer lists
    offsets: np.ndarray         # [list_off[-1]] int32, vertical offset of every entry

    def column_starts(self, d1: int) -> np.ndarray:
        return self.first[d1][:, 0, 0].copy()


def number_mixed(counts, n_layers: int, dofs, cell_vertex, cell_edge=None) -> MixedNumbering:
    lib = _lib()
    dofs = [np.ascontiguousarray(np.asarray(d, dtype=np.int32).reshape(int(counts[k]), 2)) for k, d in enumerate(dofs)]
    first = [np.full((int(counts[d]), n_layers + 1, 2), -1, dtype=np.int64) for d in range(3)]
    cnt = np.asarray(counts, dtype=np.int32)
    n_dofs = lib.oracle_alg1_number_mixed(_ptr(cnt), n_layers, _ptr(dofs[0]), _ptr(dofs[1]), _ptr(dofs[2]),
                                          _ptr(first[0]), _ptr(first[1]), _ptr(first[2]))
    cv = np.ascontiguousarray(cell_vertex, dtype=np.int32)
    ce = None if cell_edge is None else np.ascontiguousarray(cell_edge, dtype=np.int32)
    n2 = int(counts[2])
    off = np.zeros(n2 + 1, dtype=np.int64)
    total = lib.oracle_stencil_mixed(n2, n_layers, _ptr(dofs[0]), _ptr(dofs[1]), _ptr(dofs[2]), _ptr(cv), _ptr(ce),
                                     _ptr(first[0]), _ptr(first[1]), _ptr(first[2]), _ptr(off), None, None)
    lmap = np.zeros(total, dtype=np.int64)
    offsets = np.zeros(total, dtype=np.int32)
    lib.oracle_stencil_mixed(n2, n_layers, _ptr(dofs[0]), _ptr(dofs[1]), _ptr(dofs[2]), _ptr(cv), _ptr(ce),
                             _ptr(first[0]), _ptr(first[1]), _ptr(first[2]), _ptr(off), _ptr(lmap), _ptr(offsets))
    return MixedNumbering(tuple(int(x) for x in counts), n_layers, dofs, int(n_dofs), first, off, lmap, offsets)


def mixed_dg_mass(mesh, n_layers: int, vertex_coords: np.ndarray, cell_ndof, x: np.ndarray, absf: bool = False):
    """y = M x on the mixed-degree DG space whose cell c carries DG0 x DG0
    (cell_ndof[c] = 1) or DG1 x DG1 (6), numbered by number_mixed.  DG columns
    are independent, so on the DG0 cells y is the DG0 mass action of those
    cells and on the DG1 cells the DG1 one: par_loop over each cell subset on
    the uniform space of that degree, carried between the two numberings DoF
    by DoF.  Returns (y, numbering)."""
    cell_ndof = np.asarray(cell_ndof, dtype=np.int32)
    dofs = [np.zeros((mesh.n_vertices, 2), np.int32), np.zeros((mesh.n_edges, 2), np.int32),
            np.stack([np.zeros_like(cell_ndof), cell_ndof], axis=1)]
    num = number_mixed(mesh.counts, n_layers, dofs, mesh.cell_vertex, mesh.cell_edge)
    y = np.zeros(num.n_dofs)
    x = np.asarray(x, dtype=np.float64)
    lay = np.arange(n_layers)
    for name, k in (("DG0", 1), ("DG1", 6)):
        cells = np.nonzero(cell_ndof == k)[0]
        if cells.size == 0:
            continue
        pr = Problem(mesh, n_layers, name, vertex_coords)
        pos = lay[None, :, None] * k + np.arange(k)[None, None, :]
        mix = (num.lmap[num.list_off[cells]][:, None, None] + pos).ravel()
        uni = (pr.num_v.lmap[cells, 0][:, None, None] + pos).ravel()
        xu = np.zeros(pr.n_dofs)
        xu[uni] = x[mix]
        yu = pr.mass_abs(xu, cells=cells) if absf else pr.mass(xu, cells=cells)
        y[mix] = yu[uni]
    return y, num


def coordinate_field(num_x: Numbering, vertex_coords: np.ndarray) -> np.ndarray:
    """Place coords[v, l, :] of the extruded vertices at the DoFs of the P1 x P1
    coordinate space: X[dof(v, l), :]."""
    nv, nl, _ = vertex_coords.shape
    X = np.zeros((num_x.n_dofs, 3))
    dof = num_x.first[0][:, :, 0]          # [N0, lam+1]; -1 at levels outside a column (variable layers)
    used = dof.ravel() >= 0
    X[dof.ravel()[used]] = vertex_coords.reshape(-1, 3)[used]
    return X


# ---------------------------------------------------------------------------
# Algorithm 3 with the element kernels

def par_loop(form: int, space: tuple, num_v: Numbering, num_x: Numbering, X: np.ndarray,
             ins, outs, write: bool = False, cells=None, rule=None):
    """Run Algorithm 3 over all base cells (or the given subset) for one form.

    ins / outs: lists of FP64 vectors on space V (outs are updated in place:
    assigned when ``write`` else incremented)."""
    h, v = space
    lib = _lib()
    pts, wts = rule if rule is not None else rule_for(form, h, v)
    phiv = np.ascontiguousarray(tabulate(h, v, pts))
    phix, dphix = tabulate_coords(pts)
    assert phiv.shape[1] == num_v.k
    ins = list(ins) + [None] * (3 - len(ins))
    outs = list(outs) + [None] * (3 - len(outs))
    for a in ins + outs:
        if a is not None:
            assert a.dtype == np.float64 and a.flags.c_contiguous and a.size == num_v.n_dofs
    Xc = np.ascontiguousarray(X, dtype=np.float64)
    if cells is None:
        n_iter, cptr = num_v.counts[2], None
    else:
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        n_iter, cptr = cells.size, _ptr(cells)
    lib.oracle_par_loop(form, n_iter, cptr, num_v.n_layers, _ptr(num_v.cell_lam),
                        _ptr(num_x.lmap), _ptr(num_x.offsets), _ptr(Xc),
                        num_v.k, _ptr(num_v.lmap), _ptr(num_v.offsets),
                        _ptr(ins[0]), _ptr(ins[1]), _ptr(ins[2]),
                        _ptr(outs[0]), _ptr(outs[1]), _ptr(outs[2]), 1 if write else 0,
                        int(wts.size), _ptr(np.ascontiguousarray(wts)), _ptr(np.ascontiguousarray(phix)),
                        _ptr(np.ascontiguousarray(dphix)), _ptr(phiv))
    return outs


def greedy_colour(cell_vertex: np.ndarray, n_vertices: int):
    """The oracle's own greedy base-cell colouring (for timing it on several
    threads): colour [n_cells] and the number of colours; cells of one colour
    share no vertex."""
    cv = np.ascontiguousarray(cell_vertex, dtype=np.int32)
    colour = np.zeros(cv.shape[0], dtype=np.int32)
    n = _lib().oracle_greedy_colour(cv.shape[0], int(n_vertices), _ptr(cv), _ptr(colour))
    if n < 0:
        raise MemoryError("oracle_greedy_colour")
    return colour, n


def par_loop_threaded(form: int, space: tuple, num_v: Numbering, num_x: Numbering, X: np.ndarray, ins, outs,
                      write: bool = False, threads: int = 1, colour=None):
    """par_loop on several host threads, for timing the oracle on all cores:
    the same C routine on disjoint cell subsets at once (ctypes releases the
    GIL).  DG outputs (``write``) belong to one cell each, so the cells are
    simply split; increments into shared columns go colour by colour
    (``colour`` from greedy_colour), each colour's cells split over the
    threads.  The values equal par_loop's up to the order of summation."""
    from concurrent.futures import ThreadPoolExecutor
    h, v = space
    lib = _lib()
    pts, wts = rule_for(form, h, v)
    phiv = np.ascontiguousarray(tabulate(h, v, pts))
    phix, dphix = tabulate_coords(pts)
    wts, phix, dphix = (np.ascontiguousarray(a) for a in (wts, phix, dphix))
    ins = list(ins) + [None] * (3 - len(ins))
    outs = list(outs) + [None] * (3 - len(outs))
    Xc = np.ascontiguousarray(X, dtype=np.float64)
    n_cells = int(num_v.counts[2])
    if write:
        groups = [np.arange(n_cells, dtype=np.int64)]
    else:
        assert colour is not None and colour.size == n_cells
        order = np.argsort(colour, kind="stable").astype(np.int64)
        bounds = np.searchsorted(colour[order], np.arange(int(colour.max()) + 2))
        groups = [order[bounds[k]:bounds[k + 1]] for k in range(bounds.size - 1)]

    def run(cells):
        lib.oracle_par_loop(form, cells.size, _ptr(cells), num_v.n_layers, _ptr(num_v.cell_lam),
                            _ptr(num_x.lmap), _ptr(num_x.offsets), _ptr(Xc),
                            num_v.k, _ptr(num_v.lmap), _ptr(num_v.offsets),
                            _ptr(ins[0]), _ptr(ins[1]), _ptr(ins[2]),
                            _ptr(outs[0]), _ptr(outs[1]), _ptr(outs[2]), 1 if write else 0,
                            int(wts.size), _ptr(wts), _ptr(phix), _ptr(dphix), _ptr(phiv))

    with ThreadPoolExecutor(max_workers=threads) as ex:
        for g in groups:
            parts = [np.ascontiguousarray(p) for p in np.array_split(g, threads) if p.size]
            list(ex.map(run, parts))   # one colour at a time
    return outs


def _cell_subset(num_v, cells):
    if cells is None:
        return int(num_v.counts[2]), None, None
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    return cells.size, cells, _ptr(cells)


def assemble(form: int, space: tuple, num_v: Numbering, num_x: Numbering, X: np.ndarray, u=None, cells=None):
    """Matrix of a bilinear form on V (ASM_*), as scipy CSR with sorted
    indices: oracle_assemble's triplets, one per (prism, p, j) in Algorithm 3's
    order, summed per (row, column) by scipy's COO-to-CSR conversion.  Every
    pair of DoFs that share a prism is present, even where the sum is zero."""
    import scipy.sparse as sps
    h, v = space
    if num_v.cell_lam is not None:
        raise ValueError("assembly takes meshes with one layer count")
    jac = form in (ASM_CUBIC_JAC, ASM_CUBIC_JAC_ABS)
    pts, wts = rule_for(FORM_CUBIC_JVP if jac else FORM_MASS, h, v)
    phiv = np.ascontiguousarray(tabulate(h, v, pts))
    phix, dphix = tabulate_coords(pts)
    k = num_v.k
    n_iter, cells, cptr = _cell_subset(num_v, cells)
    m = n_iter * num_v.n_layers * k * k
    rows = np.empty(m, np.int64)
    cols = np.empty(m, np.int64)
    vals = np.empty(m, np.float64)
    if jac:
        assert u is not None and u.dtype == np.float64 and u.size == num_v.n_dofs
        u = np.ascontiguousarray(u)
    _lib().oracle_assemble(form, n_iter, cptr, num_v.n_layers, _ptr(num_x.lmap), _ptr(num_x.offsets),
                           _ptr(np.ascontiguousarray(X, dtype=np.float64)), k, _ptr(num_v.lmap),
                           _ptr(num_v.offsets), _ptr(u) if jac else None, _ptr(rows), _ptr(cols), _ptr(vals),
                           int(wts.size), _ptr(np.ascontiguousarray(wts)), _ptr(np.ascontiguousarray(phix)),
                           _ptr(np.ascontiguousarray(dphix)), _ptr(phiv))
    n = num_v.n_dofs
    A = sps.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def facet_loop(space: tuple, num_v: Numbering, num_x: Numbering, X: np.ndarray, x: np.ndarray,
               absf: bool = False, cells=None) -> np.ndarray:
    """Algorithm 3 over the horizontal facets (lambda + 1 per column):
    y_i = sum over facets of the integral of [x][v_i] dS, [w] the value below
    minus the value above (zero outside the domain).  The triangle rule is
    exact for the product of two horizontal basis functions (the surface
    element of a facet is constant: the map of each level is affine)."""
    h, v = space
    if num_v.cell_lam is not None:
        raise ValueError("the facet loop takes meshes with one layer count")
    n_tri = max(1, (2 * _DEG_H[h] + 2) // 2)
    tp, tw = triangle_rule(n_tri)
    nq = tp.shape[0]
    psix = np.stack([1.0 - tp[:, 0] - tp[:, 1], tp[:, 0], tp[:, 1]], axis=1)
    dpsix = np.tile(np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]]), (nq, 1, 1))
    lo = np.ascontiguousarray(tabulate(h, v, np.column_stack([tp, np.ones(nq)])))
    hi = np.ascontiguousarray(tabulate(h, v, np.column_stack([tp, np.zeros(nq)])))
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.size == num_v.n_dofs
    y = np.zeros(num_v.n_dofs)
    n_iter, cells, cptr = _cell_subset(num_v, cells)
    _lib().oracle_facet_loop(n_iter, cptr, num_v.n_layers, _ptr(num_x.lmap), _ptr(num_x.offsets),
                             _ptr(np.ascontiguousarray(X, dtype=np.float64)), num_v.k, _ptr(num_v.lmap),
                             _ptr(num_v.offsets), _ptr(x), _ptr(y), 1 if absf else 0, nq,
                             _ptr(np.ascontiguousarray(tw)), _ptr(np.ascontiguousarray(psix)),
                             _ptr(np.ascontiguousarray(dpsix)), _ptr(lo), _ptr(hi))
    return y


# ---------------------------------------------------------------------------
# Convenience wrappers for the forms of the hot path

SPACES = {
    "P1": ("CG1", "CG1"),
    "DG0": ("DG0", "DG0"),
    "DG1": ("DG1", "DG1"),
    "P2": ("CG2", "CG2"),
    "CG1xDG0": ("CG1", "DG0"),
    "CG1xDG1": ("CG1", "DG1"),
    "DG0xCG1": ("DG0", "CG1"),
    "DG0xDG1": ("DG0", "DG1"),
    "DG1xCG1": ("DG1", "CG1"),
    "DG1xDG0": ("DG1", "DG0"),
}


def is_continuous(space: tuple) -> bool:
    return space[0].startswith("CG") or space[1].startswith("CG")


class Problem:
    """A base mesh extruded to n_layers with its coordinate field and one space."""

    def __init__(self, mesh, n_layers: int, space: str | tuple, vertex_coords: np.ndarray, layers=None):
        self.mesh = mesh
        self.n_layers = n_layers
        self.space = SPACES.get(space, space) if isinstance(space, str) else space
        counts = mesh.counts
        self.num_x = number(counts, n_layers, delta_table("CG1", "CG1"), mesh.cell_vertex, mesh.cell_edge, layers)
        self.num_v = number(counts, n_layers, delta_table(*self.space), mesh.cell_vertex, mesh.cell_edge, layers)
        self.X = coordinate_field(self.num_x, vertex_coords)

    @property
    def n_dofs(self) -> int:
        return self.num_v.n_dofs

    def mass(self, x, cells=None):
        """y = M x, i.e. the residual y_i = integral of x_h v_i (Section 4.1.1)."""
        y = np.zeros(self.n_dofs)
        par_loop(FORM_MASS, self.space, self.num_v, self.num_x, self.X, [x], [y],
                 write=not is_continuous(self.space), cells=cells)
        return y

    def cubic(self, u, f, cells=None):
        F = np.zeros(self.n_dofs)
        par_loop(FORM_CUBIC, self.space, self.num_v, self.num_x, self.X, [u, f], [F], cells=cells)
        return F

    def cubic_vjp(self, u, w, cells=None):
        gu = np.zeros(self.n_dofs)
        gf = np.zeros(self.n_dofs)
        par_loop(FORM_CUBIC_VJP, self.space, self.num_v, self.num_x, self.X, [u, w], [gu, gf], cells=cells)
        return gu, gf

    def cubic_jvp(self, u, du, df, cells=None):
        dF = np.zeros(self.n_dofs)
        par_loop(FORM_CUBIC_JVP, self.space, self.num_v, self.num_x, self.X, [u, du, df], [dF], cells=cells)
        return dF

    def facet_jump(self, x, cells=None):
        """y_i = sum over horizontal facets of integral [x][v_i] dS (the
        facet loop, lambda + 1 facets per column)."""
        return facet_loop(self.space, self.num_v, self.num_x, self.X, x, cells=cells)

    def facet_jump_abs(self, x, cells=None):
        return facet_loop(self.space, self.num_v, self.num_x, self.X, x, absf=True, cells=cells)

    def mass_matrix(self, cells=None):
        """M_ij = integral phi_j phi_i (scipy CSR), from the prisms of all
        base cells or of the given ones."""
        return assemble(ASM_MASS, self.space, self.num_v, self.num_x, self.X, cells=cells)

    def mass_matrix_abs(self, cells=None):
        return assemble(ASM_MASS_ABS, self.space, self.num_v, self.num_x, self.X, cells=cells)

    def cubic_jacobian(self, u):
        """J_ij = d F_i / d u_j = integral 3 u^2 phi_j phi_i (P1 x P1, scipy CSR)."""
        return assemble(ASM_CUBIC_JAC, self.space, self.num_v, self.num_x, self.X, u)

    def cubic_jacobian_abs(self, u):
        return assemble(ASM_CUBIC_JAC_ABS, self.space, self.num_v, self.num_x, self.X, u)

    def mass_abs(self, x, cells=None):
        """Integral of |x_h| |v_i| with |.| on every factor: the scale of the
        rounding error of any summation order of mass(x)."""
        y = np.zeros(self.n_dofs)
        par_loop(FORM_MASS_ABS, self.space, self.num_v, self.num_x, self.X, [x], [y],
                 write=not is_continuous(self.space), cells=cells)
        return y

    def cubic_abs(self, u, f, cells=None):
        y = np.zeros(self.n_dofs)
        par_loop(FORM_CUBIC_ABS, self.space, self.num_v, self.num_x, self.X, [u, f], [y], cells=cells)
        return y

    def vjp_abs(self, u, w, cells=None):
        a = np.zeros(self.n_dofs)
        b = np.zeros(self.n_dofs)
        par_loop(FORM_VJP_ABS, self.space, self.num_v, self.num_x, self.X, [u, w], [a, b], cells=cells)
        return a, b

    def cubic_fused(self, u, f, w, cells=None):
        F = np.zeros(self.n_dofs)
        gu = np.zeros(self.n_dofs)
        gf = np.zeros(self.n_dofs)
        par_loop(FORM_CUBIC_FUSED, self.space, self.num_v, self.num_x, self.X, [u, f, w], [F, gu, gf], cells=cells)
        return F, gu, gf
