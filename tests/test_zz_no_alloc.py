"""The allocation-free CSR export against exm_matrix_csr, through the C ABI:
two calls in a row, the second on a smaller matrix, each bit-exact against
the allocating export (integers and the copied values alike)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1604_05937_amd as exm
from paper_1604_05937_amd import _abi, meshgen
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


def _csr(A, fn):
    rowptr = torch.full((A.n_rows + 1,), -7, dtype=torch.int64, device="cuda")
    col = torch.full((max(A.nnz, 1),), -7, dtype=torch.int32, device="cuda")
    val = torch.full((max(A.nnz, 1),), -7.0, dtype=torch.float64, device="cuda")
    getattr(_abi, fn)(A.handle, ctypes.c_void_p(rowptr.data_ptr()), ctypes.c_void_p(col.data_ptr()),
                      ctypes.c_void_p(val.data_ptr()), exm.stream_handle())
    torch.cuda.synchronize()
    return rowptr.cpu().numpy(), col[:A.nnz].cpu().numpy(), val[:A.nnz].cpu().numpy()


def _matrix(n, lam, space):
    base = meshgen.tri_square(n)
    mesh = exm.Mesh(base, lam)
    Vx = exm.Space(mesh, "P1")
    V = exm.Space(mesh, space) if space != "P1" else Vx
    X = exm.coordinate_field(Vx, meshgen.extruded_vertex_coords(base, lam, terrain=0.1))
    A = exm.Matrix(V)
    A.assemble(exm.EXM_K_MASS, X, Vx)
    return mesh, Vx, V, X, A


@pytest.mark.parametrize("first,second", [((40, 30, "P1"), (9, 7, "P2")), ((24, 100, "DG1"), (5, 3, "P1"))])
def test_csr_noalloc_matches_csr(first, second):
    for n, lam, space in (first, second):
        say(f"csr noalloc {n}x{n}x{lam} {space}")
        keep = _matrix(n, lam, space)
        A = keep[-1]
        want = _csr(A, "exm_matrix_csr")
        got = _csr(A, "exm_matrix_csr_noalloc")
        assert want[0][0] == 0 and want[0][-1] == A.nnz
        for w, g in zip(want, got):
            np.testing.assert_array_equal(g, w)


def test_csr_noalloc_rows_across_scan_segments():
    # more rows than one scan segment (8192) and a ragged last segment
    keep = _matrix(20, 60, "P1")
    A = keep[-1]
    assert A.n_rows > 3 * 8192 and A.n_rows % 8192
    want = _csr(A, "exm_matrix_csr")
    got = _csr(A, "exm_matrix_csr_noalloc")
    for w, g in zip(want, got):
        np.testing.assert_array_equal(g, w)
