"""GPU parity of the multigrid pieces (Sec. 6, Sec. 7) against the oracle:
level displacements, diagonals, transfers, eigenvalue estimates, Chebyshev,
V-cycle, PCG and the Newton driver, plus the host-forced error paths."""
import numpy as np
import pytest
import torch
from scipy.optimize import brentq

import workloads as W
from oracle import fe, gmg
from paper_1904_13131_amd import F32, F64, MfhError
from tests.gpu_helpers import dev, host, log_case, rel_l2, rel_max, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

HIER = {
    "3d_q2": dict(dim=3, n_coarse=2, degree=2, n_levels=3, spheres=3, amp=0.01),
    "2d_q3": dict(dim=2, n_coarse=2, degree=3, n_levels=3, spheres=0, amp=0.01),
    "3d_q1": dict(dim=3, n_coarse=2, degree=1, n_levels=3, spheres=2, amp=0.01),
    # loaded states (stretch of the last axis plus a small perturbation at the node positions)
    "2d_q4_vertex": dict(dim=2, n_coarse=1, degree=4, n_levels=3, spheres=0, amp=0.0025, level_field="vertex",
                         stretch=0.05),
    "3d_q3_vertex": dict(dim=3, n_coarse=1, degree=3, n_levels=3, spheres=2, amp=0.0025, level_field="vertex",
                         stretch=0.05),
    # the paper's coarse solver: Chebyshev iteration reducing the residual by 10^3
    "3d_q2_chebcoarse": dict(dim=3, n_coarse=2, degree=2, n_levels=3, spheres=3, amp=0.01, coarse="chebyshev"),
}
_CACHE = {}
# Largest Lanczos Ritz value after 30 FP64 CG steps, device against oracle
# (measured up to 1.1e-15 over HIER).  The smoother and V-cycle comparisons
# below also run on the oracle's estimates, through mfh_set_level_eigenvalues.
LAMBDA_TOL = 1e-13
# FP32 V-cycle against the FP64 oracle on the same smoother intervals: a
# linear map evaluated in FP32 (unit roundoff 6e-8) through up to 16 operator
# applications per level and three levels.
VCYCLE_F32_TOL = 2e-5
# FP64 V-cycle with its own Lanczos estimates and the Chebyshev coarse solver:
# the interval starts at the coarse run's smallest Ritz value, which rounding
# alone moves far (one-ulp perturbations of the oracle's own products move
# its V-cycle by up to 6e-6:
# test_oracle_gmg.py::test_chebyshev_coarse_own_estimate_sensitivity).
CHEB_OWN_TOL = 1e-4


def _fix_intervals(P, H):
    """Hands the oracle's eigenvalue estimates to the device, so that both build
    their smoothers (and the Chebyshev coarse solver) on the same intervals."""
    for l in range(1, H.n_levels):
        P.set_level_eigenvalues(l, H.lam_max[l])
    if H.coarse_solver == "chebyshev":
        P.set_level_eigenvalues(0, H.lam_max[0], H.lam_min0)


def _setup(name):
    if name in _CACHE:
        return _CACHE[name]
    c = HIER[name]
    dim = c["dim"]
    mu, lam = W.two_phase_material()
    incl = W.spheres(c["spheres"], 3, dim) if c["spheres"] else [(np.full(dim, 0.5), 0.3, 1)]
    mask = W.clamp_bottom_top(dim)
    mat = fe.Material(mu, lam, incl)
    H = gmg.Hierarchy(dim, c["n_coarse"], c["degree"], c["n_levels"], mat, mask,
                      level_field=c.get("level_field", "nodal"), coarse_solver=c.get("coarse", "direct"))
    fine = H.meshes[-1]
    if "stretch" in c:
        u = W.stretched_field(dim, fine.L, c["stretch"], 4, c["amp"], coords=fine.coords_1d())
    else:
        u = W.sine_field(dim, fine.L, 4, c["amp"], kmax=1)
        u[H.cons[-1]] = 0.0
    H.set_deformation(u)
    b = W.normal_vector(fine.n_dofs, 5)
    b[H.cons[-1]] = 0.0
    _CACHE[name] = (c, mu, lam, incl, mask, H, u, b)
    return _CACHE[name]


def _device(name, vdt, **kw):
    from paper_1904_13131_amd import Problem
    c, mu, lam, incl, mask, H, u, b = _setup(name)
    P = Problem(c["dim"], c["n_coarse"] * 2 ** (c["n_levels"] - 1), c["degree"], n_levels=c["n_levels"],
                mu=tuple(mu), lam=tuple(lam), inclusions=incl, dirichlet_mask=mask, vcycle_dtype=vdt,
                level_field=1 if c.get("level_field") == "vertex" else 0,
                coarse_solver=1 if c.get("coarse") == "chebyshev" else 0, **kw)
    P.set_deformation(dev(u))
    return P


@pytest.mark.parametrize("name", list(HIER))
def test_level_data(name):
    log_case("level_data", name=name)
    c, mu, lam, incl, mask, H, u, b = _setup(name)
    P = _device(name, F64)
    for l in range(c["n_levels"]):
        ul = host(P.level_displacement(l))
        assert rel_l2(ul, H.us[l]) <= 1e-13
        dg = host(P.level_diagonal(l))
        assert rel_l2(dg, H.A[l].diagonal()) <= 1e-12
    for l in range(1, c["n_levels"]):
        lam_gpu = P.level_lambda_max(l)
        err = abs(lam_gpu - H.lam_max[l]) / H.lam_max[l]
        print(f"[lambda_max] {name} level {l}: rel err {err:.2e}", flush=True)
        # 30 CG steps without reorthogonalisation: the two runs' summation
        # orders differ, and the Ritz value inherits the difference
        assert err <= LAMBDA_TOL


@pytest.mark.parametrize("dtype", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("name", list(HIER))
def test_transfers(name, dtype):
    log_case("transfers", name=name, dtype=dtype)
    c, mu, lam, incl, mask, H, u, b = _setup(name)
    P = _device(name, F64)
    tdt = torch.float64 if dtype == F64 else torch.float32
    tol = 1e-14 if dtype == F64 else 2e-6
    for l in range(1, c["n_levels"]):
        xc = W.normal_vector(H.meshes[l - 1].n_dofs, 40 + l)
        xc[H.cons[l - 1]] = 0.0
        want = H.P[l] @ xc.astype(np.float32 if dtype == F32 else np.float64).astype(np.float64)
        want[H.cons[l]] = 0.0
        got = host(P.prolongate(l, dev(xc, tdt)))
        assert rel_l2(got, want) <= tol
        xf = W.normal_vector(H.meshes[l].n_dofs, 50 + l)
        want = H.P[l].T @ xf.astype(np.float32 if dtype == F32 else np.float64).astype(np.float64)
        want[H.cons[l - 1]] = 0.0
        got = host(P.restrict(l, dev(xf, tdt)))
        assert rel_l2(got, want) <= tol


@pytest.mark.parametrize("name", list(HIER))
def test_chebyshev_and_vcycle_fp64(name):
    """On the oracle's smoother intervals the FP64 Chebyshev smoother and the
    FP64 V-cycle agree with the oracle to rounding (1e-12 relative, and the
    largest entry error against the largest entry)."""
    log_case("cheb_vcycle_f64", name=name)
    c, mu, lam, incl, mask, H, u, b = _setup(name)
    P = _device(name, F64)
    _fix_intervals(P, H)
    top = c["n_levels"] - 1
    f = b.copy()
    x0 = W.normal_vector(len(b), 77) * 0.1
    x0[H.cons[-1]] = 0.0
    lo, hi = H.interval[top]
    want = gmg.chebyshev(lambda v: H.A[top] @ v, H.dinv[top], f, x0, lo, hi, H.cheb_degree)
    got = host(P.chebyshev(top, dev(f), dev(x0)))
    z, zw = host(P.gmg_vcycle(dev(b))), H.vcycle(b)
    print(f"[cheb_vcycle_f64] {name}: chebyshev rel {rel_l2(got, want):.2e} max {rel_max(got, want):.2e}, "
          f"vcycle rel {rel_l2(z, zw):.2e} max {rel_max(z, zw):.2e}", flush=True)
    assert rel_l2(got, want) <= 1e-12 and rel_max(got, want) <= 1e-12
    assert rel_l2(z, zw) <= 1e-12 and rel_max(z, zw) <= 1e-12


@pytest.mark.parametrize("cb", [0, 1], ids=["block0", "block1"])
@pytest.mark.parametrize("name", ["3d_q2", "3d_q3_vertex", "2d_q4_vertex"])
def test_vcycle_element_cell_blocks(name, cb):
    """The ELEMENT scatter on every level (Chebyshev steps fused into the node
    sums) with either cell-block length of the pencil kernels: the FP64
    V-cycle agrees with the oracle to 1e-12 on the oracle's intervals."""
    log_case("vcycle_elem_blocks", name=name, cell_block=cb)
    c, mu, lam, incl, mask, H, u, b = _setup(name)
    P = _device(name, F64, scatter=3, cell_block=cb)
    _fix_intervals(P, H)
    z, zw = host(P.gmg_vcycle(dev(b))), H.vcycle(b)
    assert rel_l2(z, zw) <= 1e-12 and rel_max(z, zw) <= 1e-12


@pytest.mark.parametrize("name", list(HIER))
def test_vcycle_fp64_own_estimates(name):
    """With its own Lanczos estimates the FP64 V-cycle still agrees with the
    oracle to 1e-12: the largest Ritz values agree to rounding (LAMBDA_TOL).
    The Chebyshev coarse solver also takes the smallest Ritz value of the
    coarse run, which 30 steps leave far from converged and sensitive to the
    summation order, and its polynomial (degree 94 here) amplifies that
    (measured 5.9e-9 and 1.2e-7 in two runs whose coarse products summed in
    different orders; CHEB_OWN_TOL); on the oracle's estimates it agrees to
    1e-12 (above)."""
    log_case("vcycle_f64_own", name=name)
    c, mu, lam, incl, mask, H, u, b = _setup(name)
    P = _device(name, F64)
    z, zw = host(P.gmg_vcycle(dev(b))), H.vcycle(b)
    dl = max(abs(P.level_lambda_max(l) - H.lam_max[l]) / H.lam_max[l] for l in range(1, c["n_levels"]))
    print(f"[vcycle_f64_own] {name}: lambda rel {dl:.2e}, vcycle rel {rel_l2(z, zw):.2e}", flush=True)
    assert rel_l2(z, zw) <= (CHEB_OWN_TOL if c.get("coarse") == "chebyshev" else 1e-12)


@pytest.mark.parametrize("name", list(HIER))
def test_vcycle_fp32(name):
    log_case("vcycle_f32", name=name)
    c, mu, lam, incl, mask, H, u, b = _setup(name)
    P = _device(name, F32)
    _fix_intervals(P, H)
    z, zw = host(P.gmg_vcycle(dev(b))), H.vcycle(b)
    print(f"[vcycle_f32] {name}: rel {rel_l2(z, zw):.2e} max {rel_max(z, zw):.2e}", flush=True)
    assert rel_l2(z, zw) <= VCYCLE_F32_TOL and rel_max(z, zw) <= VCYCLE_F32_TOL


@pytest.mark.parametrize("vdt", [F64, F32], ids=["f64", "f32"])
@pytest.mark.parametrize("name", list(HIER))
def test_cg_solve(name, vdt):
    log_case("cg", name=name, vcycle=vdt)
    c, mu, lam, incl, mask, H, u, b = _setup(name)
    P = _device(name, vdt)
    x, it, rel, st = P.cg_solve(dev(b), rtol=1e-8, max_it=200)
    xh = host(x)
    assert rel <= 1e-8
    assert np.linalg.norm(b - H.A[-1] @ xh) <= 1.05e-8 * np.linalg.norm(b)
    assert np.all(xh[H.cons[-1]] == 0.0)
    _, it_o, _ = gmg.pcg(lambda v: H.A[-1] @ v, b, H.vcycle, 1e-8, 200)
    if vdt == F64:
        assert abs(it - it_o) <= 1
    else:
        assert it <= it_o + 3


@pytest.mark.parametrize("vdt", [F64, F32], ids=["f64", "f32"])
def test_newton_uniaxial_closed_form(vdt):
    """Homogeneous cube on rollers stretched by delta: F = diag(s, s, 1+delta),
    mu s^2 = mu - 2 lambda ln(s^2 (1+delta))."""
    from paper_1904_13131_amd import Problem
    log_case("newton_uniaxial", vcycle=vdt)
    dim, delta, mu, lam = 3, 0.1, 1.0, 1.5
    ax = dim - 1
    mask = W.face_bits(dim, ax, 0, [ax]) | W.face_bits(dim, ax, 1, [ax])
    for a in range(dim - 1):
        mask |= W.face_bits(dim, a, 0, [a])
    fv = np.zeros((2 * dim, dim))
    fv[2 * ax + 1][ax] = delta
    P = Problem(dim, 8, 2, n_levels=3, mu=(mu,), lam=(lam,), dirichlet_mask=mask, vcycle_dtype=vdt)
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    recs, st = P.newton_solve(u, fv, n_steps=2)
    s = brentq(lambda s: mu * s * s - (mu - 2 * lam * np.log(s * s * (1 + delta))), 0.5, 1.5)
    m = fe.Mesh(dim, 8, 2)
    X = m.node_coords()
    want = X * np.array([s - 1, s - 1, delta])
    got = host(u).reshape(dim, -1).T
    assert np.abs(got - want).max() <= 1e-9
    assert all(r["cg_relres"] <= 1e-8 for r in recs)


@pytest.mark.parametrize("vdt", [F64, F32], ids=["f64", "f32"])
def test_newton_cutback_matches_oracle(vdt):
    """2-D plane strain with a stiff disc compressed by 30 % in one increment:
    the second Newton iterate meets negative curvature (CG breakdown), so both
    drivers halve the failed increment, twice; the converged solutions agree."""
    from paper_1904_13131_amd import Problem
    from oracle import newton
    log_case("newton_cutback", vcycle=vdt)
    mu, lam = W.two_phase_material()
    incl = [(np.array([0.5, 0.5]), 0.3, 1)]
    mask = W.clamp_bottom_top(2)
    H = gmg.Hierarchy(2, 2, 2, 3, fe.Material(mu, lam, incl), mask)
    fv = np.zeros((4, 2))
    fv[3][1] = -0.3
    u_o, recs_o = newton.solve(H, fv, n_steps=1)
    P = Problem(2, 8, 2, n_levels=3, mu=tuple(mu), lam=tuple(lam), inclusions=incl, dirichlet_mask=mask,
                vcycle_dtype=vdt)
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    recs, st = P.newton_solve(u, fv, n_steps=1)
    assert max(r["cutbacks"] for r in recs) == max(r["cutbacks"] for r in recs_o) == 2
    assert recs[-1]["load_fraction"] == 1.0
    assert rel_l2(host(u), u_o) <= 1e-7


@pytest.mark.parametrize("vdt", [F64, F32], ids=["f64", "f32"])
def test_newton_step_length_matches_oracle(vdt):
    """35 % compression in one increment: the first full step inverts a
    quadrature point, both drivers take alpha = 1/2, carry the rest of the
    prescribed values in the next step, cut back twice and converge to the
    same state."""
    from paper_1904_13131_amd import Problem
    from oracle import newton
    log_case("newton_step_length", vcycle=vdt)
    mu, lam = W.two_phase_material()
    incl = [(np.array([0.5, 0.5]), 0.3, 1)]
    mask = W.clamp_bottom_top(2)
    H = gmg.Hierarchy(2, 2, 2, 3, fe.Material(mu, lam, incl), mask)
    fv = np.zeros((4, 2))
    fv[3][1] = -0.35
    u_o, recs_o = newton.solve(H, fv, n_steps=1)
    P = Problem(2, 8, 2, n_levels=3, mu=tuple(mu), lam=tuple(lam), inclusions=incl, dirichlet_mask=mask,
                vcycle_dtype=vdt)
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    recs, st = P.newton_solve(u, fv, n_steps=1)
    assert st == 0
    assert recs[0]["step_length"] == recs_o[0]["alpha"] == 0.5
    assert max(r["cutbacks"] for r in recs) == max(r["cutbacks"] for r in recs_o)
    assert recs[-1]["load_fraction"] == 1.0
    # CG iteration counts differ by one now and then (summation order), which
    # can move a Newton step's convergence test by one step
    assert abs(len(recs) - len(recs_o)) <= (2 if vdt == F64 else 6)
    assert rel_l2(host(u), u_o) <= 1e-8


def test_newton_q4_200_spheres_coarsest_level_matches_oracle():
    """The Q4 body of 200 spheres (seed 7) at its coarsest resolution (3^3
    cells, one level: the preconditioner is the exact coarse solve), clamped
    and compressed 20 % in 5 load steps (Sec. 7 load stepping): every load
    step converges on both sides with the same Newton steps, to the same
    state."""
    from paper_1904_13131_amd import Problem
    from oracle import newton
    log_case("newton_q4_200_spheres_3cube")
    mu, lam = W.two_phase_material()
    incl = W.spheres(200, 7, 3)
    mask = W.clamp_bottom_top(3)
    H = gmg.Hierarchy(3, 3, 4, 1, fe.Material(mu, lam, incl), mask)
    fv = np.zeros((6, 3))
    fv[5][2] = -0.2
    u_o, recs_o = newton.solve(H, fv, n_steps=5)
    P = Problem(3, 3, 4, n_levels=1, mu=tuple(mu), lam=tuple(lam), inclusions=incl, dirichlet_mask=mask,
                vcycle_dtype=F64, qp_policy=2)
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    recs, st = P.newton_solve(u, fv, n_steps=5)
    assert st == 0
    assert [r["load_fraction"] for r in recs] == [r["load_fraction"] for r in recs_o]
    assert all(r["step_length"] == 1.0 for r in recs)
    assert rel_l2(host(u), u_o) <= 1e-10
    assert abs(recs[-1]["min_J"] - fe.min_jacobian(H.meshes[-1], H.us[-1])) <= 1e-8


def test_coarse_inertia_matches_oracle():
    """A hydrostatically compressed clamped body has an indefinite tangent; the
    exact coarse solve counts its negative eigenvalues (pivot signs)."""
    from paper_1904_13131_amd import Problem
    log_case("coarse_inertia")
    mask = W.clamp_bottom_top(3)
    m = fe.Mesh(3, 2, 2)
    X = m.node_coords()
    u = np.ascontiguousarray((-0.15 * X).T.reshape(-1))
    cons = m.constrained(mask)
    K = fe.constrain_matrix(fe.tangent_matrix(m, fe.Material([1.0], [1.5]), u), cons).toarray()
    ev = np.linalg.eigvalsh(K)
    want = int((ev < 0).sum())
    kappa = np.abs(ev).max() / np.abs(ev).min()
    assert want > 0
    P = Problem(3, 2, 2, n_levels=1, mu=(1.0,), lam=(1.5,), dirichlet_mask=mask, vcycle_dtype=F64)
    P.set_deformation(dev(u))
    assert P.coarse_inertia() == want
    b = W.normal_vector(P.n_dofs(), 3)
    b[cons] = 0.0
    z = host(P.gmg_vcycle(dev(b)))            # one level: the V-cycle is the exact solve
    # the solve multiplies by an explicitly inverted matrix (Gauss-Jordan), whose
    # residual is bounded by a modest multiple of n u kappa, not u kappa; the
    # matrix entries themselves are summed by atomics, so the rounding varies
    n_free = int((~cons).sum())
    assert rel_l2(K @ z, b) <= n_free * np.finfo(np.float64).eps * kappa


def test_error_paths():
    from paper_1904_13131_amd import Problem
    log_case("errors")
    c, mu, lam, incl, mask, H, u, b = _setup("3d_q2")
    P = _device("3d_q2", F32)
    # CG iteration limit
    with pytest.raises(MfhError) as e:
        P.cg_solve(dev(b), rtol=1e-12, max_it=1)
    assert e.value.name == "NOT_CONVERGED"
    x, it, rel, st = P.cg_solve(dev(b), rtol=1e-12, max_it=1, raise_on_error=False)
    assert it == 1 and rel > 0
    # NaN right-hand side -> breakdown, detected before any iteration
    bn = b.copy()
    bn[5] = np.nan
    with pytest.raises(MfhError) as e:
        P.cg_solve(dev(bn), rtol=1e-8, max_it=10)
    assert e.value.name == "BREAKDOWN"
    # inverted element
    ui = u.copy()
    nn = len(u) // 3
    fine = H.meshes[-1]
    X = fine.node_coords()
    ui[:nn] = -3.0 * X[:, 0]          # F_xx = -2 everywhere
    with pytest.raises(MfhError) as e:
        P.set_deformation(dev(ui))
    assert e.value.name == "INVERTED"
    with pytest.raises(MfhError) as e:
        P.tangent_vmult(dev(b))
    assert e.value.name == "INVALID_ARG"
    # the problem is usable again after a good deformation
    P.set_deformation(dev(u))
    y = host(P.tangent_vmult(dev(b)))
    assert rel_l2(y, H.A[-1] @ b) <= 1e-12
    # an unconstrained compressed coarse level: singular (translations) and indefinite
    Pc = Problem(3, 2, 1, n_levels=1, mu=(1.0,), lam=(1.5,))
    mc = fe.Mesh(3, 2, 1)
    Xc = mc.node_coords()
    uc = np.ascontiguousarray((-0.7 * Xc).T.reshape(-1))
    assert Pc.set_deformation(dev(uc)) > 0
    with pytest.raises(MfhError) as e:
        Pc.cg_solve(dev(np.ones(Pc.n_dofs())), rtol=1e-8, max_it=5)
    assert e.value.name == "NOT_SPD"


def test_eigenvalue_reuse():
    """eig_refresh = 0 keeps the first linearisation's estimates (and the
    smoother built from them) for later ones; 1 recomputes them each time."""
    from paper_1904_13131_amd import Problem
    log_case("eig_reuse")
    c, mu, lam, incl, mask, H, u, b = _setup("3d_q2")
    for refresh in (0, 1):
        P = _device("3d_q2", F64, eig_refresh=refresh)
        lam1 = [P.level_lambda_max(l) for l in (1, 2)]
        P.set_deformation(dev(0.5 * u))
        lam2 = [P.level_lambda_max(l) for l in (1, 2)]
        if refresh == 0:
            assert lam2 == lam1
        else:
            assert all(abs(a - b_) > 1e-12 * a for a, b_ in zip(lam1, lam2))
        x, it, rel, st = P.cg_solve(dev(b), rtol=1e-8, max_it=200)
        assert rel <= 1e-8


@pytest.mark.parametrize("dim,n,p", [(3, 4, 2), (2, 5, 3), (3, 3, 4), (2, 6, 1)])
def test_external_force_matches_oracle(dim, n, p):
    from paper_1904_13131_amd import Problem
    log_case("external_force", dim=dim, n=n, p=p)
    mask = W.clamp_bottom_top(dim) if dim == 3 else W.face_bits(dim, 1, 0)
    ft = np.zeros((2 * dim, dim))
    ft[2 * (dim - 1) + 1] = np.linspace(0.3, -0.2, dim)        # top face
    ft[1][0] = 0.7                                              # x = 1 face, normal component
    P = Problem(dim, n, p, dirichlet_mask=mask)
    f = host(P.external_force(ft))
    m = fe.Mesh(dim, n, p)
    want = fe.external_force(m, ft)
    want[m.constrained(mask)] = 0.0
    assert np.abs(f - want).max() <= 1e-14 * np.abs(want).max()


@pytest.mark.parametrize("vdt", [F64, F32], ids=["f64", "f32"])
def test_newton_traction_closed_form(vdt):
    """Dead traction t on the top face of a cube on rollers: F = diag(s, s,
    1 + delta) with P_zz = t and no lateral stress, exactly representable."""
    from scipy.optimize import fsolve

    from paper_1904_13131_amd import Problem
    log_case("newton_traction", vcycle=vdt)
    dim, t, mu, lam = 3, 0.08, 1.0, 1.5
    mask = W.face_bits(dim, 2, 0, [2]) | W.face_bits(dim, 0, 0, [0]) | W.face_bits(dim, 1, 0, [1])
    ft = np.zeros((6, 3))
    ft[5][2] = t
    P = Problem(dim, 8, 2, n_levels=3, mu=(mu,), lam=(lam,), dirichlet_mask=mask, vcycle_dtype=vdt)
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    recs, st = P.newton_solve(u, np.zeros((6, 3)), n_steps=2, face_traction=ft)

    def eqs(v):
        s, d = v
        c1 = mu - 2 * lam * np.log(s * s * (1 + d))
        return [mu * s * s - c1, (mu * (1 + d) ** 2 - c1) / (1 + d) - t]
    s, d = fsolve(eqs, [1.0, 0.05], xtol=1e-14)
    X = fe.Mesh(dim, 8, 2).node_coords()
    want = X * np.array([s - 1, s - 1, d])
    assert np.abs(host(u).reshape(dim, -1).T - want).max() <= 1e-9
    assert all(r["cg_relres"] <= 1e-8 for r in recs)


def test_newton_shear_traction_matches_oracle():
    """The paper's load path on a small heterogeneous body: bottom clamped,
    shear traction on the top face in load steps (Sec. 7)."""
    from paper_1904_13131_amd import Problem
    from oracle import newton
    log_case("newton_shear")
    mu, lam = W.two_phase_material()
    incl = [(np.array([0.5, 0.5]), 0.3, 1)]
    mask = W.face_bits(2, 1, 0)
    ft = np.zeros((4, 2))
    ft[3][0] = 0.15
    H = gmg.Hierarchy(2, 2, 2, 3, fe.Material(mu, lam, incl), mask)
    u_o, recs_o = newton.solve(H, np.zeros((4, 2)), n_steps=3, face_traction=ft)
    P = Problem(2, 8, 2, n_levels=3, mu=tuple(mu), lam=tuple(lam), inclusions=incl, dirichlet_mask=mask,
                vcycle_dtype=F64)
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    recs, st = P.newton_solve(u, np.zeros((4, 2)), n_steps=3, face_traction=ft)
    assert len(recs) == len(recs_o)
    assert rel_l2(host(u), u_o) <= 1e-8
    assert np.abs(host(u)).max() > 0.05        # a visible shear deformation


@pytest.mark.parametrize("name", ["3d_q2", "2d_q4_vertex", "3d_q3_vertex"])
def test_smoother_fused_with_element_node_sums(name):
    """Every level on the ELEMENT scatter, so each Chebyshev step runs fused
    into the node-sum kernel: smoother, V-cycle (FP64) and CG (FP32 V-cycle)
    still match the oracle."""
    log_case("fused_cheb", name=name)
    c, mu, lam, incl, mask, H, u, b = _setup(name)
    P = _device(name, F64, scatter=3)
    top = c["n_levels"] - 1
    assert all(P.scatter_mode(l, F64) == 3 for l in range(c["n_levels"]))
    f = b.copy()
    x0 = W.normal_vector(len(b), 78) * 0.1
    x0[H.cons[-1]] = 0.0
    _fix_intervals(P, H)
    lo, hi = H.interval[top]
    want = gmg.chebyshev(lambda v: H.A[top] @ v, H.dinv[top], f, x0, lo, hi, H.cheb_degree)
    got = host(P.chebyshev(top, dev(f), dev(x0)))
    assert rel_l2(got, want) <= 1e-12 and rel_max(got, want) <= 1e-12
    z, zw = host(P.gmg_vcycle(dev(b))), H.vcycle(b)
    assert rel_l2(z, zw) <= 1e-12 and rel_max(z, zw) <= 1e-12
    Q = _device(name, F32, scatter=3)
    x, it, rel, _ = Q.cg_solve(dev(b), rtol=1e-8, max_it=200)
    assert rel <= 1e-8
    assert np.linalg.norm(b - H.A[-1] @ host(x)) <= 1.05e-8 * np.linalg.norm(b)


def test_newton_q2_16cube_matches_oracle_golden():
    """The 64^3 Newton benchmark's recipe at 16^3 Q2 cells (107,811 DoFs,
    levels 4^3..16^3, 20 spheres, bottom/top clamped, 10 % stretch in 4 load
    steps; Sec. 7 settings): the device's FP64 GMG-CG Newton solve against the
    oracle's, stored by tests/golden/make_newton_q2_16cube.py (oracle only).
    Same Newton steps, CG iterations within one, the same displacements."""
    import json
    import os

    from paper_1904_13131_amd import Problem
    log_case("newton_q2_16cube_golden")
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "newton_q2_16cube.json")))
    w = W.cube_spheres_q2(g["n_cells"])
    P = Problem(3, g["n_cells"], g["degree"], n_levels=g["n_levels"], mu=tuple(w["mu"]), lam=tuple(w["lam"]),
                inclusions=w["inclusions"], dirichlet_mask=W.clamp_bottom_top(3), vcycle_dtype=F64, qp_policy=2)
    assert P.n_dofs() == g["n_dofs"]
    u = torch.zeros(P.n_dofs(), dtype=torch.float64, device="cuda")
    fv = np.zeros((6, 3))
    fv[5][2] = g["stretch"]
    recs, st = P.newton_solve(u, fv, n_steps=g["n_steps"])
    assert st == 0
    assert [(r["load_fraction"], r["newton_iter"]) for r in recs] == \
        [(r["load_fraction"], r["newton"]) for r in g["records"]]
    ours, theirs = [r["cg_iters"] for r in recs], [r["cg_iters"] for r in g["records"]]
    print(f"[newton_q2_16cube] CG iterations device {ours} oracle {theirs}", flush=True)
    # FP64 CG on the same operator and preconditioner (V-cycles agree to 1e-13):
    # the counts drift apart by rounding in the later Newton steps, whose
    # right-hand sides are four to ten orders smaller
    assert all(abs(a - b) <= max(2, 0.1 * b) for a, b in zip(ours, theirs))
    uh = host(u)
    rows = np.array(g["rows"])
    err = np.abs(uh[rows] - np.array(g["u_rows"])).max() / np.abs(g["u_rows"]).max()
    print(f"[newton_q2_16cube] u rows max rel {err:.2e}, |u| {np.linalg.norm(uh):.12f} vs {g['u_norm']:.12f}",
          flush=True)
    assert err <= 1e-8
    assert abs(np.linalg.norm(uh) - g["u_norm"]) <= 1e-8 * g["u_norm"]


@pytest.mark.parametrize("n_fine,degree,n_levels,spheres,seed", [(64, 2, 5, 20, 3), (24, 4, 4, 200, 7)],
                         ids=["q2_64cube", "q4_24cube"])
def test_level_displacements_full_size(n_fine, degree, n_levels, spheres, seed):
    """The benchmark hierarchies at large size (the Newton benchmark's 64^3 Q2
    fine level with levels 4^3 .. 64^3; the 200-sphere Q4 body at 24^3 with
    levels 3^3 .. 24^3, where the support points do not nest and every
    coarse value is a weighted sum of fine ones; bottom and top clamped): the
    device's level displacements (nodal interpolation, Sec. 6) agree with the
    oracle's Kronecker-product interpolation on every level to 1e-13."""
    from paper_1904_13131_amd import Problem
    mask = W.clamp_bottom_top(3)
    w = W.problem(3, n_fine, degree, n_spheres=spheres, sphere_seed=seed, u_seed=4, u_amp=0.1 if degree == 2 else 0.02,
                  u_kmax=1, x_seed=5, mask=mask)
    mat = fe.Material(w["mu"], w["lam"], w["inclusions"])
    H = gmg.Hierarchy(3, n_fine >> (n_levels - 1), degree, n_levels, mat, mask)
    log_case("level_displacements_full", n_dofs=H.meshes[-1].n_dofs, degree=degree)
    us = H.level_displacements(w["u"])
    P = Problem(3, n_fine, degree, n_levels=n_levels, mu=tuple(w["mu"]), lam=tuple(w["lam"]),
                inclusions=w["inclusions"], dirichlet_mask=mask, qp_policy=2)
    P.set_deformation(dev(w["u"]))
    for l in range(n_levels):
        err = rel_l2(host(P.level_displacement(l)), us[l])
        print(f"[level_displacements_full] Q{degree} level {l}: rel {err:.2e}", flush=True)
        assert err <= 1e-13
    P.close()
