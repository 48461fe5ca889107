"""Pins for the oracle's discrete residual and tangent (eq. weak_form,
eq. tangent, eq. algebraic_tangent): derivative consistency, symmetry,
the small-strain limit, rigid-body and homogeneous-deformation identities."""
import numpy as np
import pytest

import workloads as W
from oracle import fe, material

CASES = [(2, 4, 1), (2, 3, 2), (3, 2, 2), (2, 2, 4), (3, 2, 1)]


def _setup(dim, N, p, amp=0.05, spheres=2, seed=4):
    m = fe.Mesh(dim, N, p)
    mu, lam = W.two_phase_material()
    incl = W.spheres(spheres, 3, dim) if spheres else []
    mat = fe.Material(mu, lam, incl)
    u = W.sine_field(dim, m.L, seed, amp, kmax=2) if amp else np.zeros(m.n_dofs)
    return m, mat, u


@pytest.mark.parametrize("dim,N,p", CASES)
def test_tangent_is_derivative_of_residual(dim, N, p):
    m, mat, u = _setup(dim, N, p)
    K = fe.tangent_matrix(m, mat, u)
    v = W.normal_vector(m.n_dofs, 11)
    eps = 1e-6
    fd = (fe.residual(m, mat, u + eps * v) - fe.residual(m, mat, u - eps * v)) / (2 * eps)
    Kv = K @ v
    assert np.linalg.norm(fd - Kv) / np.linalg.norm(Kv) < 1e-8


@pytest.mark.parametrize("dim,N,p", CASES)
def test_tangent_symmetric(dim, N, p):
    m, mat, u = _setup(dim, N, p)
    K = fe.tangent_matrix(m, mat, u)
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()


def _linear_elastic(m, mu, lam2):
    """Independent small-strain assembler: K = sum B^T D B with engineering
    (Voigt) strains and Lame pair (mu, lam2)."""
    d = m.d
    pairs = [(0, 0), (1, 1)] if d == 2 else [(0, 0), (1, 1), (2, 2)]
    pairs += [(0, 1)] if d == 2 else [(1, 2), (0, 2), (0, 1)]
    nv = len(pairs)
    D = np.zeros((nv, nv))
    for a in range(d):
        for b in range(d):
            D[a, b] = lam2
        D[a, a] += 2 * mu
    for s in range(d, nv):
        D[s, s] = mu
    nd = d * m.nA
    K = np.zeros((m.n_dofs, m.n_dofs))
    for e in range(m.n_cells):
        dofs = m.cell_dofs([e])[0]               # (d, nA)
        Ke = np.zeros((nd, nd))
        for q in range(m.nQ):
            B = np.zeros((nv, nd))
            for a in range(m.nA):
                g = m.G[q, a]
                for s, (i, j) in enumerate(pairs):
                    if i == j:
                        B[s, i * m.nA + a] = g[i]
                    else:
                        B[s, i * m.nA + a] = g[j]
                        B[s, j * m.nA + a] = g[i]
            Ke += m.W[q] * B.T @ D @ B
        idx = dofs.reshape(-1)
        K[np.ix_(idx, idx)] += Ke
    return K


@pytest.mark.parametrize("dim,N,p", [(2, 3, 2), (3, 2, 1), (3, 1, 2)])
def test_zero_deformation_is_linear_elasticity(dim, N, p):
    m, _, _ = _setup(dim, N, p, amp=0)
    mat = fe.Material([1.7], [0.9])
    K = fe.tangent_matrix(m, mat, np.zeros(m.n_dofs)).toarray()
    np.testing.assert_allclose(K, _linear_elastic(m, 1.7, 2 * 0.9), atol=1e-12 * abs(K).max())
    np.testing.assert_allclose(fe.residual(m, mat, np.zeros(m.n_dofs)), 0.0, atol=1e-15)


def _rotation(dim, th=0.6):
    if dim == 2:
        return np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    a = np.array([1.0, 2.0, -0.5]) / np.sqrt(5.25)
    Kx = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx


def _nodal(m, field):
    """Nodal vector from a per-node (n_nodes, d) array."""
    return np.ascontiguousarray(field.T.reshape(-1))


@pytest.mark.parametrize("dim,N,p", CASES)
def test_rigid_body_identities(dim, N, p):
    m, mat, u = _setup(dim, N, p)
    X = m.node_coords()
    K = fe.tangent_matrix(m, mat, u)
    # translations are in the kernel of the tangent, for any u
    for c in range(dim):
        t = np.zeros((m.n_nodes, dim))
        t[:, c] = 1.0
        assert np.abs(K @ _nodal(m, t)).max() < 1e-10 * abs(K).max()
    # finite rotations produce no residual
    Q = _rotation(dim)
    urot = _nodal(m, X @ (Q - np.eye(dim)).T)
    assert np.abs(fe.residual(m, mat, urot)).max() < 1e-12
    # infinitesimal rotation of the current configuration: K [W x] = W R node-wise
    rng = np.random.default_rng(1)
    Wm = rng.standard_normal((dim, dim))
    Wm = Wm - Wm.T
    x = X + u.reshape(dim, -1).T
    lhs = K @ _nodal(m, x @ Wm.T)
    R = fe.residual(m, mat, u).reshape(dim, -1).T
    rhs = _nodal(m, R @ Wm.T)
    assert np.linalg.norm(lhs - rhs) <= 1e-10 * np.linalg.norm(rhs)
    # and the residual sums to zero per component
    np.testing.assert_allclose(fe.residual(m, mat, u).reshape(dim, -1).sum(axis=1), 0.0, atol=1e-12)


@pytest.mark.parametrize("dim,N,p", [(2, 3, 2), (3, 2, 2), (2, 2, 3)])
def test_homogeneous_deformation_forces(dim, N, p):
    """u = (F0 - I) X on a homogeneous body: interior nodal forces vanish and
    sum_a R_(a,i) X_(a,k) = P_ik(F0) * volume, with P from the printed
    Kirchhoff stress, P = tau F^-T."""
    m, _, _ = _setup(dim, N, p, amp=0)
    mu, lam = 0.8, 1.9
    mat = fe.Material([mu], [lam])
    rng = np.random.default_rng(3)
    F0 = np.eye(dim) + 0.2 * rng.standard_normal((dim, dim))
    X = m.node_coords()
    u = _nodal(m, X @ (F0 - np.eye(dim)).T)
    R = fe.residual(m, mat, u).reshape(dim, -1).T            # (n_nodes, d)
    P = material.tau_closed_form(F0, np.float64(mu), np.float64(lam)) @ np.linalg.inv(F0).T
    np.testing.assert_allclose(R.T @ X, P, atol=1e-12)
    interior = np.all((X > 1e-12) & (X < 1 - 1e-12), axis=1)
    assert np.abs(R[interior]).max() < 1e-12


def test_rows_and_ebe_match_csr():
    m, mat, u = _setup(3, 3, 2)
    cons = m.constrained(W.clamp_bottom_top(3))
    x = W.normal_vector(m.n_dofs, 2)
    K = fe.constrain_matrix(fe.tangent_matrix(m, mat, u), cons)
    y = K @ x
    np.testing.assert_allclose(fe.vmult_ebe(m, mat, u, x, cons), y, rtol=0, atol=1e-12 * abs(y).max())
    rows = np.array([0, 7, 101, m.n_dofs // 2, m.n_dofs - 1])
    np.testing.assert_allclose(fe.vmult_rows(m, mat, u, x, rows, cons), y[rows], atol=1e-12 * abs(y).max())
    R = fe.residual(m, mat, u, cons)
    np.testing.assert_allclose(fe.residual_rows(m, mat, u, rows, cons), R[rows], atol=1e-14)
    assert np.all(R[cons] == 0)
    # identity rows and columns on constrained DoFs
    Kd = K.toarray()
    np.testing.assert_array_equal(Kd[np.ix_(cons, cons)], np.eye(cons.sum()))
    assert np.all(Kd[np.ix_(cons, ~cons)] == 0) and np.all(Kd[np.ix_(~cons, cons)] == 0)


def test_diagonal_closed_form():
    """diag K for DoF (a, alpha) = sum_q w_q h^d [c1 (|v|^2 + v_alpha^2)
    + 2 lambda v_alpha^2 + v . tau v] with v = F^-T Grad N_a (from the
    spatial form of the tangent with the printed tau and J*c)."""
    m, mat, u = _setup(3, 2, 2)
    K = fe.tangent_matrix(m, mat, u)
    F = fe.deformation_gradient(m, u, m.all_cells())
    mu, lam = mat.params(m, m.all_cells())
    tau = material.tau_closed_form(F, mu, lam)
    c1 = mu - 2 * lam * np.log(np.linalg.det(F))
    v = np.einsum("cqIj,qaI->cqaj", np.linalg.inv(F), m.G)      # v_j = Finv_Ij dN_a/dX_I
    vv = (v ** 2).sum(-1)
    tv = np.einsum("cqaj,cqjk,cqak->cqa", v, tau, v)
    diag = np.zeros(m.n_dofs)
    dofs = m.cell_dofs(m.all_cells())
    for al in range(3):
        va = v[..., al] ** 2
        val = np.einsum("q,cqa->ca", m.W, c1[..., None] * (vv + va) + 2 * lam[..., None] * va + tv)
        np.add.at(diag, dofs[:, al, :].reshape(-1), val.reshape(-1))
    np.testing.assert_allclose(diag, K.diagonal(), rtol=1e-12)


def test_square_disc_q1_16_shapes():
    c = W.square_disc_q1_16()
    m = fe.Mesh(c["dim"], c["n_cells"], c["degree"])
    assert m.n_dofs == 578
    K = fe.tangent_matrix(m, fe.Material(c["mu"], c["lam"], c["inclusions"]), c["u"])
    assert K.nnz == 9604
    assert fe.min_jacobian(m, c["u"]) > 0


# --- Mooney-Rivlin law (second law, tensor4 route) ---

def _mr_setup(dim, N, p, amp=0.05, seed=4):
    m, mat, u = _setup(dim, N, p, amp=amp, seed=seed)
    return m, fe.Material(mat.mu, mat.lam, mat.inclusions, mu2=W.two_phase_mu2()), u


@pytest.mark.parametrize("dim,N,p", [(2, 3, 2), (3, 2, 2), (3, 2, 1)])
def test_mr_tangent_is_derivative_of_residual(dim, N, p):
    m, mat, u = _mr_setup(dim, N, p)
    K = fe.tangent_matrix(m, mat, u)
    v = W.normal_vector(m.n_dofs, 12)
    eps = 1e-6
    fd = (fe.residual(m, mat, u + eps * v) - fe.residual(m, mat, u - eps * v)) / (2 * eps)
    Kv = K @ v
    assert np.linalg.norm(fd - Kv) / np.linalg.norm(Kv) < 1e-8
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()
    # the second-invariant term changes the operator
    K0 = fe.tangent_matrix(m, fe.Material(mat.mu, mat.lam, mat.inclusions), u)
    assert abs(K - K0).max() > 1e-3 * abs(K0).max()


@pytest.mark.parametrize("dim,N,p", [(2, 3, 2), (3, 2, 2)])
def test_mr_homogeneous_deformation_forces(dim, N, p):
    """As for the Neo-Hookean law, with P = tau F^-T from the law's spatial
    closed form."""
    m, _, _ = _setup(dim, N, p, amp=0)
    mu, lam, mu2 = 0.8, 1.9, 0.35
    mat = fe.Material([mu], [lam], mu2=[mu2])
    rng = np.random.default_rng(5)
    F0 = np.eye(dim) + 0.2 * rng.standard_normal((dim, dim))
    X = m.node_coords()
    u = _nodal(m, X @ (F0 - np.eye(dim)).T)
    R = fe.residual(m, mat, u).reshape(dim, -1).T
    P = material.mr_tau_closed_form(F0, np.float64(mu), np.float64(lam), np.float64(mu2)) @ np.linalg.inv(F0).T
    np.testing.assert_allclose(R.T @ X, P, atol=1e-12)
    interior = np.all((X > 1e-12) & (X < 1 - 1e-12), axis=1)
    assert np.abs(R[interior]).max() < 1e-12


# --- smallest Jacobian (Sec. 2.1: J = det F > 0 at every quadrature point) ---

def _first_gauss_point(q):
    """Smallest q-point Gauss-Legendre abscissa on [0, 1], closed forms of the
    Legendre roots (P_2: 1/sqrt(3); P_3: sqrt(3/5); P_4: sqrt(3/7 + 2/7 sqrt(6/5)))."""
    t = {2: 1 / np.sqrt(3), 3: np.sqrt(3 / 5), 4: np.sqrt(3 / 7 + 2 / 7 * np.sqrt(6 / 5))}[q]
    return 0.5 * (1 - t)


@pytest.mark.parametrize("dim,N,p", [(2, 3, 1), (3, 2, 2), (2, 2, 3), (3, 2, 1)])
def test_min_jacobian_affine_is_det_F0(dim, N, p):
    """u = (F0 - I) X is represented exactly at every degree: every quadrature
    point carries J = det F0, so the minimum is det F0 (one inverted F0 too)."""
    m = fe.Mesh(dim, N, p)
    X = m.node_coords()
    rng = np.random.default_rng(11)
    for k in range(3):
        F0 = np.eye(dim) + 0.3 * rng.standard_normal((dim, dim))
        if k == 2:
            F0[0] *= -1                                             # det F0 < 0
        u = _nodal(m, X @ (F0 - np.eye(dim)).T)
        assert abs(fe.min_jacobian(m, u) - np.linalg.det(F0)) <= 1e-13


@pytest.mark.parametrize("dim,N,p", [(2, 3, 2), (3, 2, 2), (2, 2, 3), (3, 3, 3)])
def test_min_jacobian_quadratic_field(dim, N, p):
    """u_x = a x^2, u_y = b y^2 (exact for p >= 2): F = diag(1 + 2ax, 1 + 2by, 1),
    J = (1 + 2ax)(1 + 2by).  With a, b > 0 the minimum sits at the quadrature
    point nearest the origin (x = y = h g_0, g_0 the first Gauss abscissa on
    [0, 1]); with a < 0 < b at the largest x and the smallest y."""
    m = fe.Mesh(dim, N, p)
    X = m.node_coords()
    h, g0 = 1.0 / N, _first_gauss_point(p + 1)
    lo, hi = h * g0, 1 - h * g0
    for a, b, xs, ys in [(0.3, 0.2, lo, lo), (-0.35, 0.25, hi, lo)]:
        f = np.zeros_like(X)
        f[:, 0] = a * X[:, 0] ** 2
        f[:, 1] = b * X[:, 1] ** 2
        want = (1 + 2 * a * xs) * (1 + 2 * b * ys)
        assert abs(fe.min_jacobian(m, _nodal(m, f)) - want) <= 1e-13


def test_oracle_host_spmv_matches_scipy():
    """The oracle's OpenMP CSR product (CPU baseline) computes K x."""
    from oracle import spmv
    m, mat, u = _setup(3, 3, 2)
    K = fe.tangent_matrix(m, mat, u)
    x = W.normal_vector(m.n_dofs, 3)
    y = spmv.spmv(spmv.prepare(K), x)
    assert np.linalg.norm(y - K @ x) <= 1e-14 * np.linalg.norm(K @ x)
