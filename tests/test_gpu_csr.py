"""GPU parity of the matrix-based baseline: K_c assembled on the device in CSR
form (eq. algebraic_tangent with the constraints of Sec. 3) and the CSR SpMV,
against the oracle's assembled matrix and against the matrix-free vmult.

Bar: assembled values within 1e-12 of the largest entry (FP64 sums in another
order); the pattern of every free row is exactly the set of DoFs of the cells
that hold its node (the oracle's element-by-element assembly pattern), every
constrained row is its unit diagonal; SpMV relative l2 error <= 1e-12.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads as W
from oracle import fe
from tests.gpu_helpers import dev, device_problem, host, log_case, oracle_problem, rel_l2, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

CLAMP3 = W.clamp_bottom_top(3)

CASES = {
    "square_16x16_q1": W.square_disc_q1_16(),
    "2d_q3_clamp": W.problem(2, 5, 3, disc=True, u_amp=0.04, u_kmax=2, mask=W.clamp_bottom_top(2)),
    "3d_q1_clamp": W.problem(3, 5, 1, n_spheres=3, u_amp=0.05, u_kmax=2, mask=CLAMP3),
    "3d_q2_mixedmask": W.problem(3, 3, 2, n_spheres=2, u_amp=0.05, u_kmax=2,
                                 mask=W.face_bits(3, 0, 0, [0]) | W.face_bits(3, 1, 1, [1, 2]) | W.face_bits(3, 2, 0)),
    "3d_q4_clamp": W.problem(3, 2, 4, n_spheres=2, u_amp=0.04, u_kmax=2, mask=CLAMP3),
    "3d_q3_free": W.problem(3, 3, 3, n_spheres=3, u_amp=0.04, u_kmax=2),
}


def _to_scipy(csr, n):
    rp, col, val = (t.cpu().numpy() for t in csr)
    return sp.csr_matrix((val, col.astype(np.int64), rp), shape=(n, n))


@pytest.mark.parametrize("name", list(CASES))
def test_csr_matches_oracle(name):
    log_case("csr_assemble", name=name)
    w = CASES[name]
    mesh, mat, cons = oracle_problem(w)
    K = fe.tangent_matrix(mesh, mat, w["u"])
    Kc = fe.constrain_matrix(K, cons)
    P = device_problem(w)
    P.set_deformation(dev(w["u"]))
    n, nnz = P.csr_size()
    assert n == mesh.n_dofs
    csr = P.csr_assemble()
    A = _to_scipy(csr, n)
    assert A.nnz == nnz and A.has_sorted_indices
    # pattern: free rows as the oracle's element-by-element assembly, constrained rows their diagonal
    K.sort_indices()
    free = np.nonzero(~cons)[0]
    for r in range(n):
        cols = A.indices[A.indptr[r]:A.indptr[r + 1]]
        if cons[r]:
            assert list(cols) == [r]
        else:
            assert np.array_equal(cols, K.indices[K.indptr[r]:K.indptr[r + 1]]), r
    assert np.all(A.diagonal()[cons] == 1.0)
    scale = abs(Kc).max()
    assert abs(A - Kc).max() <= 1e-12 * scale
    # SpMV against the oracle and against the matrix-free vmult
    x = w["x"]
    y = host(P.csr_spmv(csr, dev(x)))
    assert rel_l2(y, Kc @ x) <= 1e-12
    ymf = host(P.tangent_vmult(dev(x)))
    assert rel_l2(y, ymf) <= 1e-12
    assert len(free) > 0


def test_csr_coarse_level_matches_matrix_free():
    """On every level of a hierarchy the CSR SpMV equals the matrix-free vmult
    of that level (the level's own displacement field)."""
    w = W.problem(3, 8, 2, n_spheres=3, u_amp=0.03, u_kmax=1, mask=CLAMP3)
    log_case("csr_levels")
    P = device_problem(w, n_levels=3)
    P.set_deformation(dev(w["u"]))
    for level in range(3):
        n, _ = P.csr_size(level)
        x = dev(W.normal_vector(n, 40 + level))
        y = host(P.csr_spmv(P.csr_assemble(level), x, level=level))
        assert rel_l2(y, host(P.tangent_vmult(x, level=level))) <= 1e-12, level


def test_csr_q2_32cube():
    """32^3 Q2 (823,875 DoFs, the size of the operator benchmark): SpMV equals
    the matrix-free vmult, sampled rows equal the oracle's rows, and the row
    lengths match the closed form (3 * prod of per-axis node ranges)."""
    w = W.cube_spheres_q2()
    log_case("csr_q2_32cube")
    mesh, mat, cons = oracle_problem(w)
    P = device_problem(w)
    u = dev(w["u"])
    P.set_deformation(u)
    csr = P.csr_assemble()
    n, nnz = P.csr_size()
    x = dev(w["x"])
    y = P.csr_spmv(csr, x)
    ymf = P.tangent_vmult(x)
    assert rel_l2(host(y), host(ymf)) <= 1e-12
    rng = np.random.default_rng(5)
    rows = np.concatenate([rng.choice(mesh.n_dofs, 40, replace=False), np.nonzero(cons)[0][:4]])
    yo = fe.vmult_rows(mesh, mat, w["u"], w["x"], rows, constrained=cons)
    np.testing.assert_allclose(host(y)[rows], yo, rtol=0, atol=1e-12 * np.abs(yo).max())
    # row lengths in closed form: per axis 2p+1 nodes at an interior cell vertex, p+1 inside a cell,
    # p+1 on the boundary
    rp = csr[0].cpu().numpy()
    L, p = mesh.L, mesh.p
    ln = np.array([p + 1 if (I % p) or I in (0, L - 1) else 2 * p + 1 for I in range(L)])
    lat = np.indices((L,) * 3).reshape(3, -1)[::-1]
    full = 3 * ln[lat[0]] * ln[lat[1]] * ln[lat[2]]
    expect = np.where(cons, 1, np.tile(full, 3))
    assert np.array_equal(np.diff(rp), expect)
    assert rp[-1] == nnz
