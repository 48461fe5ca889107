"""Edge cases of the device path against the oracle: single-cell meshes of
every degree, fully constrained boundaries, zero and undeformed inputs, a
body that is all inclusion, the largest lattice the library accepts (2-D,
1600 nodes per direction) checked on sampled rows, 32-bit lane offsets past
2^31 and 64-bit ones past 2^32, and element-scatter cell blocks that end in
the middle of x-rows.

Bars as in the operator tests: FP64 relative l2 <= 1e-12 (absolute on
sampled rows, relative to the largest entry)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fe
from tests.gpu_helpers import dev, device_problem, host, log_case, oracle_problem, rel_l2, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

ALL_FACES = {2: (1 << 8) - 1, 3: (1 << 18) - 1}


@pytest.mark.parametrize("policy", [0, 1, 2, 3], ids=["R", "CF", "C2", "C4"])
@pytest.mark.parametrize("dim,p", [(2, 1), (2, 4), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_single_cell(dim, p, policy):
    log_case("single_cell", dim=dim, p=p, policy=policy)
    w = W.problem(dim, 1, p, disc=(dim == 2), n_spheres=0 if dim == 2 else 1, u_amp=0.03, u_kmax=1,
                  mask=W.face_bits(dim, 0, 0))
    mesh, mat, cons = oracle_problem(w)
    K = fe.constrain_matrix(fe.tangent_matrix(mesh, mat, w["u"]), cons)
    P = device_problem(w, qp_policy=policy)
    P.set_deformation(dev(w["u"]))
    y = host(P.tangent_vmult(dev(w["x"])))
    assert rel_l2(y, K @ w["x"]) <= 1e-12
    r = host(P.residual(dev(w["u"])))
    assert rel_l2(r, fe.residual(mesh, mat, w["u"], cons)) <= 1e-12


@pytest.mark.parametrize("scatter", [0, 1, 2, 3], ids=["atomic", "color", "tile", "elem"])
@pytest.mark.parametrize("dim", [2, 3])
def test_fully_constrained_boundary(dim, scatter):
    """Every face fixes every component: boundary rows are the identity (y = x
    there) and the interior rows see x with its boundary entries zeroed."""
    log_case("all_faces", dim=dim, scatter=scatter)
    w = W.problem(dim, 4 if dim == 3 else 6, 2, n_spheres=2 if dim == 3 else 0, disc=dim == 2, u_amp=0.03,
                  u_kmax=1, mask=ALL_FACES[dim])
    mesh, mat, cons = oracle_problem(w)
    K = fe.constrain_matrix(fe.tangent_matrix(mesh, mat, w["u"]), cons)
    P = device_problem(w, scatter=scatter)
    P.set_deformation(dev(w["u"]))
    y = host(P.tangent_vmult(dev(w["x"])))
    assert np.array_equal(y[cons], w["x"][cons])
    assert rel_l2(y, K @ w["x"]) <= 1e-12
    r = host(P.residual(dev(w["u"])))
    assert np.all(r[cons] == 0.0)


@pytest.mark.parametrize("policy", [0, 2], ids=["R", "C2"])
def test_zero_input_and_undeformed_state(policy):
    """K x = 0 for x = 0 (every scatter path writes every entry); at u = 0 the
    operator is the small-strain one (oracle at u = 0) and the residual is 0."""
    log_case("zero_and_undeformed", policy=policy)
    w = W.problem(3, 5, 2, n_spheres=3, u_amp=0.0, mask=W.clamp_bottom_top(3))
    mesh, mat, cons = oracle_problem(w)
    K0 = fe.constrain_matrix(fe.tangent_matrix(mesh, mat, np.zeros(mesh.n_dofs)), cons)
    for scatter in (0, 1, 2, 3):
        P = device_problem(w, qp_policy=policy, scatter=scatter)
        assert P.set_deformation(dev(np.zeros(mesh.n_dofs))) == 1.0
        y = torch.full((mesh.n_dofs,), float("nan"), dtype=torch.float64, device="cuda")
        P.tangent_vmult(dev(np.zeros(mesh.n_dofs)), y)
        assert not host(y).any()
        assert rel_l2(host(P.tangent_vmult(dev(w["x"]))), K0 @ w["x"]) <= 1e-12
        assert not host(P.residual(dev(np.zeros(mesh.n_dofs)))).any()


def test_body_that_is_all_inclusion():
    """One inclusion covering the whole body: the operator is the stiff
    material's, i.e. 100 times the matrix material's (both moduli scale)."""
    log_case("all_inclusion")
    w = W.problem(3, 3, 2, u_amp=0.04, u_kmax=1)
    w["inclusions"] = [(np.full(3, 0.5), 2.0, 1)]
    mesh, mat, cons = oracle_problem(w)
    K = fe.tangent_matrix(mesh, mat, w["u"])
    soft = fe.tangent_matrix(mesh, fe.Material([w["mu"][0]], [w["lam"][0]]), w["u"])
    assert abs(K - 100.0 * soft).max() <= 1e-11 * abs(K).max()
    P = device_problem(w)
    P.set_deformation(dev(w["u"]))
    assert rel_l2(host(P.tangent_vmult(dev(w["x"]))), K @ w["x"]) <= 1e-12


def test_largest_lattice_2d():
    """2-D Q1 with 1599 cells per direction: 1600 nodes per direction, the
    largest lattice the descriptor accepts (5.12 M DoFs); sampled rows
    (corners, edges, interior) against the oracle's row-wise vmult, and
    translations in the kernel of the unconstrained operator."""
    log_case("largest_2d")
    w = W.problem(2, 1599, 1, disc=True, u_amp=0.02, u_kmax=1)
    mesh, mat, cons = oracle_problem(w)
    assert mesh.L == 1600
    P = device_problem(w)
    P.set_deformation(dev(w["u"]))
    y = host(P.tangent_vmult(dev(w["x"])))
    L = mesh.L
    rng = np.random.default_rng(9)
    rows = np.unique(np.concatenate([rng.choice(mesh.n_dofs, 40, replace=False),
                                     [0, L - 1, L * (L - 1), L * L - 1, L * L + L // 2, 2 * L * L - 1]]))
    ref = fe.vmult_rows(mesh, mat, w["u"], w["x"], rows)
    np.testing.assert_allclose(y[rows], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    t = np.concatenate([np.ones(L * L), np.zeros(L * L)])
    assert np.abs(host(P.tangent_vmult(dev(t)))).max() <= 1e-9


def test_level_beyond_32bit_lane_offsets():
    """3-D Q1 with 350^3 cells (129 M DoFs).  The vmult addresses its per-lane
    arrays with 32-bit byte offsets when NV * cells * 2 * word < 2^32 (the
    factor 2 for the arrays of word pairs of the cache_T2 data), else with
    64-bit ones.  Here FP64 takes the 64-bit form and FP32 the 32-bit form
    with pair offsets beyond the signed range (between 2^31 and 2^32).  Both
    agree with the recompute policy on the atomic scatter over the whole
    vector and with the oracle on sampled rows."""
    from paper_1904_13131_amd import F32
    n = 350
    log_case("large_offsets", cells=n ** 3)
    w = W.problem(3, n, 1, n_spheres=20, u_amp=0.05, u_kmax=1, n_modes=2)
    assert 8 * n ** 3 * 2 * 8 >= 2 ** 32 > 8 * n ** 3 * 2 * 4 >= 2 ** 31
    mesh, mat, cons = oracle_problem(w)
    u, x = dev(w["u"]), dev(w["x"])
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([rng.integers(0, mesh.n_dofs, 16), [mesh.n_dofs - 1]]))
    ref = fe.vmult_rows(mesh, mat, w["u"], w["x"], rows)
    P = device_problem(w, qp_policy=0, scatter=0)
    P.set_deformation(u)
    y_ref = P.tangent_vmult(x)
    torch.cuda.synchronize()
    del P
    torch.cuda.empty_cache()
    Q = device_problem(w, qp_policy=2, scatter=3, vcycle_dtype=F32)
    Q.set_deformation(u)
    y = Q.tangent_vmult(x)
    torch.cuda.synchronize()
    assert float((y - y_ref).norm() / y_ref.norm()) <= 1e-12
    yh = host(y)
    np.testing.assert_allclose(yh[rows], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    y32 = Q.tangent_vmult(x.float())
    assert float((y32.double() - y_ref).norm() / y_ref.norm()) <= 1e-5


@pytest.mark.parametrize("dim,n,p", [(2, 13, 1), (2, 10, 2), (2, 9, 3), (2, 8, 4), (3, 3, 4), (3, 6, 2), (3, 5, 3)],
                         ids=["2d_q1", "2d_q2", "2d_q3", "2d_q4", "3d_q4", "3d_q2", "3d_q3"])
@pytest.mark.parametrize("policy", [0, 2], ids=["R", "C2"])
def test_element_buffer_block_ends(dim, n, p, policy):
    """Element scatter where cell blocks end in the middle of x-rows, so that
    both routes of a shared x-face node are taken: summed by the x-neighbour
    in the same block, and through the overflow part across block ends (and
    on the x = 1 face).  FP64 against the oracle's assembled tangent, FP32 to
    the FP32 bar."""
    from paper_1904_13131_amd import F32
    log_case("element_block_ends", dim=dim, n=n, p=p, policy=policy)
    w = W.problem(dim, n, p, disc=dim == 2, n_spheres=0 if dim == 2 else 3, u_amp=0.04, u_kmax=1,
                  mask=W.face_bits(dim, dim - 1, 0))
    mesh, mat, cons = oracle_problem(w)
    K = fe.constrain_matrix(fe.tangent_matrix(mesh, mat, w["u"]), cons)
    ref = K @ w["x"]
    P = device_problem(w, qp_policy=policy, scatter=3, vcycle_dtype=F32)
    P.set_deformation(dev(w["u"]))
    assert rel_l2(host(P.tangent_vmult(dev(w["x"]))), ref) <= 1e-12
    y32 = P.tangent_vmult(dev(w["x"]).float())
    assert rel_l2(host(y32.double()), K @ host(dev(w["x"]).float().double())) <= 1e-5


@pytest.mark.parametrize("degree", [3, 4])
def test_contraction_stage_forms_agree(degree):
    """The VALU and MFMA forms of the contraction stage (the autotuner's
    measurement) compute the same values: the MFMA operand layout is right."""
    import torch

    from paper_1904_13131_amd.mfh import contraction_stage
    log_case("contraction_stage", degree=degree)
    n = (degree + 1) * 256 * 8
    a = contraction_stage(degree, 0, 50, 8, torch.empty(n, dtype=torch.float32, device="cuda"))
    b = contraction_stage(degree, 1, 50, 8, torch.empty(n, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    scale = float(a.abs().max())
    assert scale > 0
    assert float((a - b).abs().max()) <= 1e-4 * scale
