"""GPU parity of the matrix-free tangent vmult and the residual (eq. mf_vmult,
eq. algebraic_tangent, eq. linear_system) against the oracle's assembled
operators, through the C ABI.

Bar: relative l2 error <= 1e-12 in FP64 and <= 1e-5 in FP32 (x rounded to
FP32 first), for every quadrature-point policy and both scatter modes.  The
small cases span several blocks of cells with a ragged last block; the full
size of the 32^3 Q2 workload (823,875 DoFs), of the 64^3 Q2 Newton level
(6,440,067 DoFs) and of the 48^3 Q4 benchmark body (21,567,171 DoFs) is
checked on sampled rows that the oracle computes one by one, plus identities
that hold at any size.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fe
from tests.gpu_helpers import dev, device_problem, host, log_case, oracle_problem, rel_l2, rel_max, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

CLAMP3 = W.clamp_bottom_top(3)
CLAMP2 = W.clamp_bottom_top(2)

CASES = {
    "square_16x16_q1": W.square_disc_q1_16(),
    "2d_q2": W.problem(2, 7, 2, disc=True, u_amp=0.04, u_kmax=2, mask=W.face_bits(2, 0, 0)),
    "2d_q3_clamp": W.problem(2, 5, 3, disc=True, u_amp=0.04, u_kmax=2, mask=CLAMP2),
    "2d_q4": W.problem(2, 4, 4, disc=True, u_amp=0.04, u_kmax=2),
    "3d_q1_clamp": W.problem(3, 5, 1, n_spheres=3, u_amp=0.05, u_kmax=2, mask=CLAMP3),
    "3d_q2": W.problem(3, 4, 2, n_spheres=3, u_amp=0.05, u_kmax=2),
    "3d_q2_mixedmask": W.problem(3, 3, 2, n_spheres=2, u_amp=0.05, u_kmax=2,
                                 mask=W.face_bits(3, 0, 0, [0]) | W.face_bits(3, 1, 1, [1, 2]) | W.face_bits(3, 2, 0)),
    "3d_q3": W.problem(3, 3, 3, n_spheres=3, u_amp=0.04, u_kmax=2),
    "3d_q4_clamp": W.problem(3, 2, 4, n_spheres=2, u_amp=0.04, u_kmax=2, mask=CLAMP3),
    # several tiles per direction (tile modes), ragged for Q3
    "3d_q4_tiles": W.problem(3, 4, 4, n_spheres=4, u_amp=0.03, u_kmax=1, mask=CLAMP3),
    "3d_q3_tiles": W.problem(3, 5, 3, n_spheres=4, u_amp=0.03, u_kmax=1, mask=CLAMP3),
}

_ORACLE = {}


def _oracle(name):
    if name not in _ORACLE:
        w = CASES[name]
        mesh, mat, cons = oracle_problem(w)
        K = fe.constrain_matrix(fe.tangent_matrix(mesh, mat, w["u"]), cons)
        R = fe.residual(mesh, mat, w["u"], cons)
        _ORACLE[name] = (mesh, mat, cons, K, R)
    return _ORACLE[name]


# (scatter mode, tile shape, cell block): both compiled tile shapes of the
# TILE scatter, both cell-block lengths of the pencil-kernel modes
SCATTERS64 = [(0, -1, 0), (0, -1, 1), (1, -1, 0), (1, -1, 1), (2, 0, 0), (2, 1, 0), (3, -1, 0), (3, -1, 1),
              (-1, -1, -1)]
SCATTERS32 = [(0, -1, 0), (0, -1, 1), (2, 0, 0), (2, 1, 0), (3, -1, 0), (3, -1, 1), (-1, -1, -1)]
IDS64 = ["atomic", "atomic_b1", "color", "color_b1", "tile0", "tile1", "elem", "elem_b1", "auto"]
IDS32 = ["atomic", "atomic_b1", "tile0", "tile1", "elem", "elem_b1", "auto"]


@pytest.mark.parametrize("scatter,tile,cb", SCATTERS64, ids=IDS64)
@pytest.mark.parametrize("policy", [0, 1, 2, 3], ids=["R", "CF", "C2", "C4"])
@pytest.mark.parametrize("name", list(CASES))
def test_vmult_fp64(name, policy, scatter, tile, cb):
    log_case("vmult_fp64", name=name, policy=policy, scatter=scatter, tile=tile, cell_block=cb)
    w = CASES[name]
    _, _, _, K, _ = _oracle(name)
    P = device_problem(w, qp_policy=policy, scatter=scatter, tile_shape=tile, cell_block=cb)
    mj = P.set_deformation(dev(w["u"]))
    assert mj > 0
    y = host(P.tangent_vmult(dev(w["x"])))
    want = K @ w["x"]
    assert rel_l2(y, want) <= 1e-12 and rel_max(y, want) <= 1e-12


@pytest.mark.parametrize("scatter,tile,cb", SCATTERS32, ids=IDS32)
@pytest.mark.parametrize("policy", [0, 1, 2, 3], ids=["R", "CF", "C2", "C4"])
@pytest.mark.parametrize("name", list(CASES))
def test_vmult_fp32(name, policy, scatter, tile, cb):
    log_case("vmult_fp32", name=name, policy=policy, scatter=scatter, tile=tile, cell_block=cb)
    w = CASES[name]
    _, _, _, K, _ = _oracle(name)
    P = device_problem(w, qp_policy=policy, scatter=scatter, tile_shape=tile, cell_block=cb)
    P.set_deformation(dev(w["u"]))
    x32 = w["x"].astype(np.float32)
    y = host(P.tangent_vmult(dev(x32, torch.float32)))
    want = K @ x32.astype(np.float64)
    assert rel_l2(y, want) <= 1e-5 and rel_max(y, want) <= 1e-5


def test_tile_shapes_reported():
    """The two compiled tile shapes of a level, forced or tuned, as reported
    by mfh_tile_shape: shape 0 of 3-D Q2 FP64 is 3 x 3 x 3 cells."""
    from paper_1904_13131_amd import F32, F64
    log_case("tile_shapes")
    w = CASES["3d_q2"]
    seen = set()
    for tile in (0, 1):
        P = device_problem(w, scatter=2, tile_shape=tile)
        for dt in (F64, F32):
            shape, cells = P.tile_shape(dtype=dt)
            assert shape == tile and len(cells) == 3 and min(cells) >= 1
            seen.add((dt, cells))
    assert (F64, (3, 3, 3)) in seen and len(seen) == 4
    P = device_problem(w, scatter=2)
    assert P.tile_shape()[0] in (0, 1)


def test_cell_blocks_reported():
    """Cells per workgroup of the two cell-block variants (3-D Q2: 27 and 14,
    3-D Q4: 8 and 10), forced and tuned, as reported by mfh_cell_block."""
    from paper_1904_13131_amd import F32, F64
    log_case("cell_blocks")
    for name, want in (("3d_q2", (27, 14)), ("3d_q4_clamp", (8, 10))):
        w = CASES[name]
        for cb in (0, 1):
            P = device_problem(w, scatter=3, cell_block=cb)
            for dt in (F64, F32):
                assert P.cell_block(dtype=dt) == (cb, want[cb])
        P = device_problem(w)
        v, cells = P.cell_block()
        assert cells == want[v]


@pytest.mark.parametrize("scatter", [0, 1], ids=["atomic", "color"])
@pytest.mark.parametrize("name", list(CASES))
def test_residual(name, scatter):
    log_case("residual", name=name, scatter=scatter)
    w = CASES[name]
    _, _, cons, _, R = _oracle(name)
    P = device_problem(w, scatter=scatter)
    r = host(P.residual(dev(w["u"])))
    assert rel_l2(r, R) <= 1e-12 and rel_max(r, R) <= 1e-12
    assert np.all(r[cons] == 0.0)


@pytest.mark.parametrize("scatter", [1, 3], ids=["color", "elem"])
def test_deterministic_scatters(scatter):
    """The colour and element scatters fix the summation order: repeated
    applications are bitwise equal (FP64 and FP32)."""
    w = CASES["3d_q2"]
    log_case("determinism", name="3d_q2", scatter=scatter)
    P = device_problem(w, scatter=scatter)
    P.set_deformation(dev(w["u"]))
    for dt in (torch.float64, torch.float32):
        x = dev(w["x"], dt)
        a = host(P.tangent_vmult(x))
        b = host(P.tangent_vmult(x))
        assert np.array_equal(a, b)


def test_min_J_matches_oracle():
    w = CASES["3d_q3"]
    log_case("minJ", name="3d_q3")
    mesh, _, _, _, _ = _oracle("3d_q3")
    P = device_problem(w)
    mj = P.set_deformation(dev(w["u"]))
    assert abs(mj - fe.min_jacobian(mesh, w["u"])) <= 1e-13


# ---- full size: 32^3 Q2, 823,875 DoFs -------------------------------------------------

_C2 = {}


def _q2_32cube():
    if not _C2:
        w = W.cube_spheres_q2()
        mesh, mat, cons = oracle_problem(w)
        rng = np.random.default_rng(17)
        rows = np.sort(rng.choice(mesh.n_dofs, 160, replace=False))
        # include lattice corners, edges and faces
        L = mesh.L
        extra = [0, L - 1, L * L - 1, mesh.n_nodes - 1, mesh.n_nodes + L * (L // 2), 2 * mesh.n_nodes + 3]
        rows = np.unique(np.concatenate([rows, extra]))
        _C2.update(w=w, mesh=mesh, mat=mat, rows=rows,
                   ref=fe.vmult_rows(mesh, mat, w["u"], w["x"], rows),
                   ref32=fe.vmult_rows(mesh, mat, w["u"], w["x"].astype(np.float32).astype(np.float64), rows),
                   rres=fe.residual_rows(mesh, mat, w["u"], rows))
    return _C2


@pytest.mark.parametrize("scatter", [0, 2, 3], ids=["atomic", "tile", "elem"])
@pytest.mark.parametrize("policy", [0, 1, 2, 3], ids=["R", "CF", "C2", "C4"])
def test_q2_32cube_sampled_rows(policy, scatter):
    c = _q2_32cube()
    w = c["w"]
    log_case("q2_32cube_rows", policy=policy, scatter=scatter, n_dofs=c["mesh"].n_dofs)
    P = device_problem(w, qp_policy=policy, scatter=scatter)
    P.set_deformation(dev(w["u"]))
    y = host(P.tangent_vmult(dev(w["x"])))
    scale = np.abs(c["ref"]).max()
    assert np.abs(y[c["rows"]] - c["ref"]).max() <= 1e-12 * scale
    y32 = host(P.tangent_vmult(dev(w["x"].astype(np.float32), torch.float32)))
    assert np.linalg.norm(y32[c["rows"]] - c["ref32"]) <= 1e-5 * np.linalg.norm(c["ref32"])
    r = host(P.residual(dev(w["u"])))
    assert np.abs(r[c["rows"]] - c["rres"]).max() <= 1e-12 * max(np.abs(c["rres"]).max(), 1e-300) + 1e-15


def test_q2_32cube_identities():
    """Translations are in the kernel of the unconstrained tangent; the
    operator is symmetric (x^T K y = y^T K x)."""
    c = _q2_32cube()
    w = c["w"]
    log_case("q2_32cube_identities")
    P = device_problem(w)
    P.set_deformation(dev(w["u"]))
    n = P.n_dofs()
    nn = n // 3
    for comp in range(3):
        t = torch.zeros(n, dtype=torch.float64, device="cuda")
        t[comp * nn:(comp + 1) * nn] = 1.0
        kt = host(P.tangent_vmult(t))
        kx = host(P.tangent_vmult(dev(w["x"])))
        assert np.abs(kt).max() <= 1e-12 * np.abs(kx).max()
    a = dev(W.normal_vector(n, 31))
    b = dev(W.normal_vector(n, 32))
    ka, kb = P.tangent_vmult(a), P.tangent_vmult(b)
    s1, s2 = float(torch.dot(b, ka)), float(torch.dot(a, kb))
    assert abs(s1 - s2) <= 1e-12 * abs(s1)


def test_q2_32cube_tangent_is_derivative_of_device_residual():
    """Central differences of the device residual along a smooth direction
    match the device tangent at full size (823,875 DoFs): the two kernels
    evaluate R and dR/du through different formulas (the first Piola stress
    against its linearisation), so this ties them together where the oracle
    cannot assemble."""
    c = _q2_32cube()
    w = c["w"]
    log_case("q2_32cube_fd")
    P = device_problem(w)
    P.set_deformation(dev(w["u"]))
    v = W.sine_field(3, c["mesh"].L, 21, 1.0, kmax=1)
    u = dev(w["u"])
    eps = 1e-5
    fd = (host(P.residual(u + eps * dev(v))) - host(P.residual(u - eps * dev(v)))) / (2 * eps)
    kv = host(P.tangent_vmult(dev(v)))
    err = rel_l2(fd, kv)
    print(f"[q2_32cube_fd] rel {err:.2e}", flush=True)
    # truncation error O(eps^2) times the third derivative, rounding O(1e-16 / eps)
    assert err <= 1e-8


# ---- full size: 48^3 Q4 with 200 spheres, 21,567,171 DoFs ----------------------------

_C4 = {}


def _q4_48cube():
    """The 48^3 Q4 body (200 spheres, seed 7, bottom and top clamped) at a
    smooth state, with sampled rows that the oracle computes one by one:
    random rows plus nodes shared by 1, 2, 4 and 8 cells and constrained ones."""
    if not _C4:
        w = W.problem(3, 48, 4, n_spheres=200, sphere_seed=7, u_seed=4, u_amp=0.02, u_kmax=1, x_seed=5,
                      mask=CLAMP3)
        mesh, mat, cons = oracle_problem(w)
        rng = np.random.default_rng(19)
        rows = rng.choice(mesh.n_dofs, 100, replace=False)
        L = mesh.L
        node = lambda i, j, k: i + L * (j + L * k)
        extra = [node(4, 4, 4), node(4, 2, 7), node(8, 8, 3), node(1, 2, 3), node(0, 96, 96),
                 node(L - 1, L - 1, 100), node(50, 60, 0), node(L - 1, 0, L - 1)]
        extra += [mesh.n_nodes + e for e in extra[:4]] + [2 * mesh.n_nodes + e for e in extra[:4]]
        rows = np.unique(np.concatenate([rows, extra]))
        _C4.update(w=w, mesh=mesh, mat=mat, cons=cons, rows=rows,
                   ref=fe.vmult_rows(mesh, mat, w["u"], w["x"], rows, constrained=cons),
                   ref32=fe.vmult_rows(mesh, mat, w["u"], w["x"].astype(np.float32).astype(np.float64), rows,
                                       constrained=cons),
                   rres=fe.residual_rows(mesh, mat, w["u"], rows, constrained=cons))
    return _C4


@pytest.mark.parametrize("policy", [0, 2], ids=["R", "C2"])
def test_q4_48cube_sampled_rows(policy):
    """The finest level of the Q4 benchmark at its real size (even-odd sweeps,
    8-cell blocks, element scatter): FP64 rows to 1e-12 of the largest entry,
    FP32 to 1e-5, residual rows to 1e-12."""
    c = _q4_48cube()
    w = c["w"]
    log_case("q4_48cube_rows", policy=policy, n_dofs=c["mesh"].n_dofs)
    P = device_problem(w, qp_policy=policy)
    P.set_deformation(dev(w["u"]))
    y = host(P.tangent_vmult(dev(w["x"])))
    scale = np.abs(c["ref"]).max()
    err = np.abs(y[c["rows"]] - c["ref"]).max() / scale
    y32 = host(P.tangent_vmult(dev(w["x"].astype(np.float32), torch.float32)))
    err32 = np.linalg.norm(y32[c["rows"]] - c["ref32"]) / np.linalg.norm(c["ref32"])
    r = host(P.residual(dev(w["u"])))
    rscale = max(np.abs(c["rres"]).max(), 1e-300)
    errr = np.abs(r[c["rows"]] - c["rres"]).max() / rscale
    print(f"[q4_48cube_rows] policy {policy}: fp64 {err:.2e} fp32 {err32:.2e} residual {errr:.2e}", flush=True)
    assert err <= 1e-12 and err32 <= 1e-5 and errr <= 1e-12
    P.close()


def test_q4_48cube_tangent_is_derivative_of_device_residual():
    """Central differences of the device residual along a smooth direction
    converge to the device tangent on the 48^3 Q4 body (constrained rows
    excluded: the tangent holds identity rows there, the residual zeros).
    The truncation error of the central difference (step squared times the
    third derivative) grows with the resolution of this 200-sphere body: the
    oracle's own difference quotient at step 1e-5 is off by 1.9e-9 at 4^3
    and 4.5e-9 at 6^3, and the device's by about 1e-6 at 48^3; so the test
    checks the second-order decay (a quarter of the step must cut the error
    about sixteenfold, which a mismatch between residual and tangent would
    not; measured 1.93e-7 at step 4e-6 and 1.21e-8 at 1e-6) and the error
    at the smaller step."""
    c = _q4_48cube()
    w = c["w"]
    log_case("q4_48cube_fd")
    P = device_problem(w, qp_policy=2)
    P.set_deformation(dev(w["u"]))
    v = W.sine_field(3, c["mesh"].L, 21, 1.0, kmax=1)
    v[c["cons"]] = 0.0
    u, dv = dev(w["u"]), dev(v)
    kv = host(P.tangent_vmult(dv))
    free = ~c["cons"]
    errs = []
    for eps in (4e-6, 1e-6):
        fd = (host(P.residual(u + eps * dv)) - host(P.residual(u - eps * dv))) / (2 * eps)
        errs.append(rel_l2(fd[free], kv[free]))
    print(f"[q4_48cube_fd] rel {errs[0]:.2e} (step 4e-6), {errs[1]:.2e} (step 1e-6)", flush=True)
    assert errs[1] <= 0.1 * errs[0] and errs[1] <= 5e-8
    P.close()


def test_q2_64cube_sampled_rows():
    """The finest level of the Newton benchmark at its real size (64^3 Q2,
    6,440,067 DoFs, 20 spheres, bottom and top clamped) on sampled rows:
    cached-F^-1 vmult FP64 to 1e-12 of the largest entry, FP32 to 1e-5,
    residual to 1e-12."""
    w = W.problem(3, 64, 2, n_spheres=20, sphere_seed=3, u_seed=4, u_amp=0.1, u_kmax=1, x_seed=5, mask=CLAMP3)
    mesh, mat, cons = oracle_problem(w)
    rng = np.random.default_rng(23)
    L = mesh.L
    node = lambda i, j, k: i + L * (j + L * k)
    extra = [node(2, 2, 2), node(64, 63, 1), node(128, 128, 64), node(7, 0, 0), node(0, 5, 128)]
    rows = np.unique(np.concatenate([rng.choice(mesh.n_dofs, 100, replace=False), extra,
                                     [mesh.n_nodes + e for e in extra], [2 * mesh.n_nodes + e for e in extra]]))
    log_case("q2_64cube_rows", n_dofs=mesh.n_dofs)
    ref = fe.vmult_rows(mesh, mat, w["u"], w["x"], rows, constrained=cons)
    ref32 = fe.vmult_rows(mesh, mat, w["u"], w["x"].astype(np.float32).astype(np.float64), rows, constrained=cons)
    rres = fe.residual_rows(mesh, mat, w["u"], rows, constrained=cons)
    P = device_problem(w, qp_policy=2)
    P.set_deformation(dev(w["u"]))
    y = host(P.tangent_vmult(dev(w["x"])))
    err = np.abs(y[rows] - ref).max() / np.abs(ref).max()
    y32 = host(P.tangent_vmult(dev(w["x"].astype(np.float32), torch.float32)))
    err32 = np.linalg.norm(y32[rows] - ref32) / np.linalg.norm(ref32)
    r = host(P.residual(dev(w["u"])))
    errr = np.abs(r[rows] - rres).max() / np.abs(rres).max()
    print(f"[q2_64cube_rows] fp64 {err:.2e} fp32 {err32:.2e} residual {errr:.2e}", flush=True)
    assert err <= 1e-12 and err32 <= 1e-5 and errr <= 1e-12
    P.close()
