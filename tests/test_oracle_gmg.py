"""Pins for the oracle's multigrid pieces (Sec. 6 transfers and level
operators; Sec. 7 Chebyshev smoother, eigenvalue estimate, PCG)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

import workloads as W
from oracle import fe, gmg, rng


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 3), (3, 2), (2, 4)])
def test_prolongation_reproduces_coarse_polynomials(dim, p):
    c, f = fe.Mesh(dim, 2, p), fe.Mesh(dim, 4, p)
    P = gmg.prolongation(c, f)
    I = gmg.interpolation(f, c)
    r = np.random.default_rng(0)
    coef = r.standard_normal((dim,) + (p + 1,) * dim)
    def field(X):
        out = np.zeros((X.shape[0], dim))
        for comp in range(dim):
            for idx in np.ndindex(*coef.shape[1:]):
                out[:, comp] += coef[(comp,) + idx] * np.prod([X[:, k] ** idx[k] for k in range(dim)], axis=0)
        return np.ascontiguousarray(out.T.reshape(-1))
    uc, uf = field(c.node_coords()), field(f.node_coords())
    np.testing.assert_allclose(P @ uc, uf, atol=1e-12)
    np.testing.assert_allclose(I @ uf, uc, atol=1e-12)
    np.testing.assert_allclose((I @ P).toarray(), np.eye(c.n_dofs), atol=1e-13)


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 1), (3, 2), (2, 3)])
def test_galerkin_identity_affine_homogeneous(dim, p):
    """P^T K_f P = K_c when u is affine and the body homogeneous: the coarse
    space is contained in the fine one and q = p+1 integrates the (polynomial)
    integrands exactly."""
    c, f = fe.Mesh(dim, 1 if dim == 3 else 2, p), fe.Mesh(dim, 2 if dim == 3 else 4, p)
    mat = fe.Material([1.1], [1.6])
    F0 = np.eye(dim) + 0.15 * np.random.default_rng(2).standard_normal((dim, dim))
    def affine(m):
        X = m.node_coords()
        return np.ascontiguousarray((X @ (F0 - np.eye(dim)).T).T.reshape(-1))
    Kc = fe.tangent_matrix(c, mat, affine(c)).toarray()
    Kf = fe.tangent_matrix(f, mat, affine(f))
    P = gmg.prolongation(c, f)
    np.testing.assert_allclose((P.T @ Kf @ P).toarray(), Kc, atol=1e-12 * abs(Kc).max())


def test_chebyshev_error_polynomial():
    """On a diagonal system D^-1 A = diag(t) with x0 = 0 and f = A e, the
    error after one degree-k application is T_k((theta - t)/delta) /
    T_k(theta/delta) e."""
    t = np.linspace(0.05, 2.0, 40)
    e = np.random.default_rng(1).standard_normal(40)
    dvals = np.linspace(1.0, 3.0, 40)
    A = t * dvals
    lo, hi = 0.6, 2.1
    for k in (1, 2, 3, 4, 6):
        x = gmg.chebyshev(lambda v: A * v, 1.0 / dvals, A * e, np.zeros(40), lo, hi, k)
        theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
        Tk = np.polynomial.chebyshev.Chebyshev.basis(k)
        want = Tk((theta - t) / delta) / Tk(theta / delta) * e
        np.testing.assert_allclose(e - x, want, atol=1e-12)


def test_lanczos_estimate_vs_dense_eigensolver():
    mu, lam = W.two_phase_material()
    m = fe.Mesh(3, 3, 2)
    mat = fe.Material(mu, lam, W.spheres(2, 3))
    cons = m.constrained(W.clamp_bottom_top(3))
    u = W.sine_field(3, m.L, 4, 0.02, kmax=1)
    A = fe.constrain_matrix(fe.tangent_matrix(m, mat, u), cons)
    dinv = 1.0 / A.diagonal()
    est, its = gmg.lanczos_lambda_max(lambda v: A @ v, dinv, gmg.eig_start_vector(m.n_dofs, cons), 30)
    s = np.sqrt(dinv)
    true = np.linalg.eigvalsh(s[:, None] * A.toarray() * s[None, :]).max()
    assert its == 30
    assert est <= true * (1 + 1e-12)
    assert est >= true * (1 - 1e-3)


def test_splitmix64_published_vectors():
    """SplitMix64 seeded with 1234567: first outputs as published with the
    reference implementation (xoshiro/splitmix64.c test vector)."""
    z = rng.splitmix64(1234567, 5)
    assert [int(v) for v in z] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                    4593380528125082431, 16408922859458223821]


def test_pcg_with_vcycle_matches_direct_solve():
    mu, lam = W.two_phase_material()
    mat = fe.Material(mu, lam, W.spheres(3, 3))
    H = gmg.Hierarchy(3, 2, 2, 2, mat, W.clamp_bottom_top(3))
    u = W.sine_field(3, H.meshes[-1].L, 4, 0.01, kmax=1)
    u[H.cons[-1]] = 0.0
    H.set_deformation(u)
    b = W.normal_vector(H.meshes[-1].n_dofs, 5)
    b[H.cons[-1]] = 0.0
    x, it, rel = gmg.pcg(lambda v: H.A[-1] @ v, b, H.vcycle, 1e-10, 200)
    xd = spl.spsolve(H.A[-1].tocsc(), b)
    assert rel <= 1e-10
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    assert np.all(x[H.cons[-1]] == 0)


def test_pcg_reports_breakdown_on_negative_curvature():
    """CG on an indefinite operator stops with a NaN relative residual at the
    first direction of non-positive curvature (p^T A p <= 0)."""
    A = np.diag([1.0, -1.0, 2.0])
    b = np.array([0.0, 1.0, 0.0])
    x, it, rel = gmg.pcg(lambda v: A @ v, b, lambda r: r.copy(), 1e-8, 10)
    assert it == 1 and np.isnan(rel) and np.all(x == 0)
    # an SPD operator with the same right-hand side converges in one step
    x, it, rel = gmg.pcg(lambda v: np.abs(A) @ v, b, lambda r: r.copy(), 1e-8, 10)
    assert it == 1 and rel == 0.0 and np.allclose(x, b)


def test_vcycle_is_symmetric_and_h_independent():
    """The V-cycle is a symmetric preconditioner, and for a homogeneous body
    the PCG iteration count does not grow under refinement (Sec. 6)."""
    mat = fe.Material([1.0], [1.5])
    counts = []
    for nl in (2, 3):
        H = gmg.Hierarchy(3, 2, 2, nl, mat, W.clamp_bottom_top(3))
        H.set_deformation(np.zeros(H.meshes[-1].n_dofs))
        n = H.meshes[-1].n_dofs
        a, b = W.normal_vector(n, 1), W.normal_vector(n, 2)
        a[H.cons[-1]] = 0
        b[H.cons[-1]] = 0
        assert abs(a @ H.vcycle(b) - b @ H.vcycle(a)) <= 1e-10 * abs(a @ H.vcycle(b))
        _, it, rel = gmg.pcg(lambda v, H=H: H.A[-1] @ v, b, H.vcycle, 1e-8, 100)
        counts.append(it)
    assert counts[1] <= counts[0] + 1
    assert counts[1] <= 15


def test_level_displacements_are_nodal_interpolants():
    mat = fe.Material([1.0], [1.5])
    H = gmg.Hierarchy(2, 2, 2, 3, mat)
    X = H.meshes[-1].node_coords()
    u = np.ascontiguousarray(np.stack([np.sin(3 * X[:, 0]) * X[:, 1], X[:, 0] ** 2], 0).reshape(-1))
    us = H.level_displacements(u)
    for l in range(3):
        Xl = H.meshes[l].node_coords()
        want = np.ascontiguousarray(np.stack([np.sin(3 * Xl[:, 0]) * Xl[:, 1], Xl[:, 0] ** 2], 0).reshape(-1))
        np.testing.assert_allclose(us[l], want, atol=1e-14)   # p = 2 nodes nest: injection


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 4), (2, 1)])
def test_vertex_level_fields(dim, p):
    """VERTEX level fields: every coarse level carries the fine field's values
    at its own cell vertices and is multilinear in each of its cells, so it
    reproduces any globally multilinear field exactly; for degree 1 it equals
    nodal interpolation."""
    mat = fe.Material([1.0], [1.5])
    H = gmg.Hierarchy(dim, 1, p, 3, mat, level_field="vertex")
    Hn = gmg.Hierarchy(dim, 1, p, 3, mat, level_field="nodal")
    fine = H.meshes[-1]
    X = fine.node_coords()
    # a globally multilinear field: reproduced on every level
    lin = np.prod(1.0 + 0.3 * X, axis=1)
    u = np.ascontiguousarray(np.stack([lin * (c + 1) for c in range(dim)], 0).reshape(-1))
    for l, ul in enumerate(H.level_displacements(u)):
        Xl = H.meshes[l].node_coords()
        want = np.ascontiguousarray(np.stack([np.prod(1.0 + 0.3 * Xl, axis=1) * (c + 1) for c in range(dim)], 0).reshape(-1))
        np.testing.assert_allclose(ul, want, atol=1e-13)
    # a smooth non-multilinear field: coarse vertex values equal the fine values there
    g = np.sin(2.0 * X[:, 0]) + np.cos(3.0 * X[:, -1]) * X[:, 0]
    u = np.ascontiguousarray(np.tile(g, dim))
    us = H.level_displacements(u)
    for l in range(2):
        m = H.meshes[l]
        Xl = m.node_coords()
        on_vertex = np.all(np.isclose((Xl * m.N) % 1.0, 0.0) | np.isclose((Xl * m.N) % 1.0, 1.0), axis=1)
        gl = np.sin(2.0 * Xl[:, 0]) + np.cos(3.0 * Xl[:, -1]) * Xl[:, 0]
        np.testing.assert_allclose(us[l][:m.n_nodes][on_vertex], gl[on_vertex], atol=1e-13)
    if p == 1:
        for a, b in zip(H.level_displacements(u), Hn.level_displacements(u)):
            np.testing.assert_allclose(a, b, atol=1e-14)


def test_chebyshev_coarse_solver():
    """Sec. 7's coarse solver: the degree follows the Chebyshev error bound,
    and one application reduces the coarse residual (in the D^-1 A energy of a
    definite operator) by at least the requested 10^3 when the interval holds
    the spectrum; with the Lanczos interval it still reduces by about that."""
    # kappa = 100: acosh(1000) = 7.6009, acosh(101/99) = 0.20067 -> 37.9; the classical
    # estimate ln(2/eps) sqrt(kappa) / 2 = 38.0 agrees
    assert gmg.chebyshev_solver_degree(1.0, 100.0, 1e-3) == 38
    # exact interval on a diagonal operator: guaranteed reduction
    rng = np.random.default_rng(0)
    lam = np.linspace(0.5, 40.0, 200)
    A = np.diag(lam)
    k = gmg.chebyshev_solver_degree(0.5, 40.0, 1e-3)
    b = rng.standard_normal(200)
    x = gmg.chebyshev(lambda v: A @ v, np.ones(200), b, np.zeros(200), 0.5, 40.0, k)
    e0, e = np.linalg.solve(A, b), np.linalg.solve(A, b) - x
    assert np.sqrt(e @ A @ e) <= 1e-3 * np.sqrt(e0 @ A @ e0) * (1 + 1e-12)
    # in the hierarchy
    mat = fe.Material([1.0], [1.5])
    H = gmg.Hierarchy(3, 2, 2, 2, mat, W.clamp_bottom_top(3), coarse_solver="chebyshev")
    H.set_deformation(np.zeros(H.meshes[-1].n_dofs))
    assert 0 < H.lam_min0 < H.lam_max[0]
    r = W.normal_vector(H.meshes[0].n_dofs, 3)
    r[H.cons[0]] = 0
    z = H.vcycle(r, 0)
    res = r - H.A[0] @ z
    assert np.linalg.norm(res) <= 0.05 * np.linalg.norm(r)
    b = W.normal_vector(H.meshes[-1].n_dofs, 5)
    b[H.cons[-1]] = 0
    _, it, rel = gmg.pcg(lambda v: H.A[-1] @ v, b, H.vcycle, 1e-8, 200)
    assert rel <= 1e-8


def test_chebyshev_coarse_own_estimate_sensitivity():
    """The Chebyshev coarse solver (Sec. 7) starts its interval at the smallest
    Ritz value of the coarse level's 30-step CG-Lanczos run, which is far from
    converged: perturbing every product of that run by one unit in the last
    place (a change of summation order does as much) moves it by 1e-7 to
    2e-4 and the whole V-cycle by 4e-9 to 6e-6 on the 3-D Q2 hierarchy of the
    device comparison (two coarse cells, three levels, three spheres), while
    the largest Ritz value stays within 1e-15.  So a device V-cycle with its
    own estimates cannot match the oracle's to 1e-12 in this configuration;
    the device test holds it to 1e-4 and the shared-interval one to 1e-12."""
    mu, lam = W.two_phase_material()
    mat = fe.Material(mu, lam, W.spheres(3, 3, 3))
    H = gmg.Hierarchy(3, 2, 2, 3, mat, W.clamp_bottom_top(3), coarse_solver="chebyshev")
    fine = H.meshes[-1]
    u = W.sine_field(3, fine.L, 4, 0.01, kmax=1)
    u[H.cons[-1]] = 0.0
    H.set_deformation(u)
    b = W.normal_vector(fine.n_dofs, 5)
    b[H.cons[-1]] = 0.0
    z0 = H.vcycle(b)
    lmin0, lmax0 = H.lam_min0, H.lam_max[0]
    A, m = H.A[0], H.meshes[0]
    rg = np.random.default_rng(1)
    dz, dmin, dmax = [], [], []
    for _ in range(12):
        def apply(v):
            y = A @ v
            return y * (1.0 + 2.0 ** -52 * rg.choice([-1.0, 1.0], size=y.shape))
        lmax, _ = gmg.lanczos_lambda_max(apply, H.dinv[0], gmg.eig_start_vector(m.n_dofs, H.cons[0]), H.eig_iters)
        lmin = gmg.lanczos_lambda_max.last_min
        H.interval[0] = (lmin, H.cheb_hi * lmax)
        H.coarse_degree = gmg.chebyshev_solver_degree(lmin, H.cheb_hi * lmax, gmg.COARSE_REDUCTION)
        z = H.vcycle(b)
        dz.append(np.linalg.norm(z - z0) / np.linalg.norm(z0))
        dmin.append(abs(lmin - lmin0) / lmin0)
        dmax.append(abs(lmax - lmax0) / lmax0)
    assert max(dmax) <= 1e-14
    assert max(dmin) >= 1e-8 and max(dz) >= 1e-9     # far above rounding
    assert max(dz) <= 1e-4                          # the device test's bar


def _spd(n, eigs, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return (q * np.asarray(eigs, dtype=np.float64)) @ q.T


def test_lanczos_extreme_ritz_values_exact_on_few_eigenvalues():
    """With k distinct eigenvalues of D^-1 A, k CG steps span the whole Krylov
    space, so the k Ritz values are those eigenvalues: both the largest
    (smoother interval) and the smallest (coarse Chebyshev solver) are exact."""
    n, dist = 24, np.array([0.7, 2.0, 5.5, 13.0])
    A = _spd(n, np.repeat(dist, n // 4), 1)
    est, its = gmg.lanczos_lambda_max(lambda v: A @ v, np.ones(n), W.normal_vector(n, 2), 4)
    assert its == 4
    assert abs(est - 13.0) <= 1e-11 * 13.0
    assert abs(gmg.lanczos_lambda_max.last_min - 0.7) <= 1e-11 * 13.0


def test_lanczos_smallest_ritz_value_full_run_and_interlacing():
    """A Jacobi-preconditioned run on a 12 x 12 SPD system with a non-trivial
    diagonal: 12 steps give the extreme eigenvalues of D^-1/2 A D^-1/2, and
    shorter runs interlace (smallest Ritz value non-increasing, never below
    the smallest eigenvalue; largest non-decreasing, never above the largest)."""
    n = 12
    B = _spd(n, np.geomspace(0.5, 40.0, n), 3)
    d = np.geomspace(1.0, 30.0, n)
    A = np.sqrt(d)[:, None] * B * np.sqrt(d)[None, :]        # D^-1/2 A D^-1/2 = B
    dinv = 1.0 / A.diagonal()
    s = np.sqrt(dinv)
    ev = np.linalg.eigvalsh(s[:, None] * A * s[None, :])
    r0 = W.normal_vector(n, 4)
    lo_prev, hi_prev = np.inf, 0.0
    for it in range(1, n + 1):
        hi, m = gmg.lanczos_lambda_max(lambda v: A @ v, dinv, r0, it)
        lo = gmg.lanczos_lambda_max.last_min
        assert m == it
        assert lo >= ev[0] * (1 - 1e-10) and hi <= ev[-1] * (1 + 1e-10)
        assert lo <= lo_prev * (1 + 1e-10) and hi >= hi_prev * (1 - 1e-10)
        lo_prev, hi_prev = lo, hi
    assert abs(lo - ev[0]) <= 1e-8 * ev[0]
    assert abs(hi - ev[-1]) <= 1e-8 * ev[-1]
