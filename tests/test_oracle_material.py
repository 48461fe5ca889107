"""Pins for the Neo-Hookean law of Sec. 2.3: derivatives by central finite
differences of the energy, and the push-forward identities of Sec. 2.1 against
the spatial closed forms the paper prints."""
import numpy as np
import pytest

from oracle import material as M

MU, LAM = 1.3, 2.1


def _F(dim, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    F = np.eye(dim) + scale * rng.standard_normal((dim, dim))
    assert np.linalg.det(F) > 0
    return F


def _fd(fun, F, h=1e-6):
    dim = F.shape[0]
    out = np.zeros(np.shape(fun(F)) + (dim, dim))
    for k in range(dim):
        for L in range(dim):
            E = np.zeros_like(F)
            E[k, L] = h
            out[..., k, L] = (fun(F + E) - fun(F - E)) / (2 * h)
    return out


@pytest.mark.parametrize("dim,seed", [(2, 0), (2, 1), (3, 2), (3, 3)])
def test_pk1_is_derivative_of_energy(dim, seed):
    F = _F(dim, seed)
    P = M.pk1(F, np.float64(MU), np.float64(LAM))
    fd = _fd(lambda G: M.psi(G, MU, LAM), F)
    np.testing.assert_allclose(P, fd, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("dim,seed", [(2, 4), (3, 5), (3, 6)])
def test_tangent_is_derivative_of_pk1(dim, seed):
    F = _F(dim, seed)
    A = M.dP_dF(F, np.float64(MU), np.float64(LAM))
    fd = _fd(lambda G: M.pk1(G, np.float64(MU), np.float64(LAM)), F)
    np.testing.assert_allclose(A, fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("dim,seed", [(2, 7), (3, 8)])
def test_referential_tangent_is_second_derivative(dim, seed):
    """CC = 4 d2psi/dC2: S(C + e dC) - S(C - e dC) = 2e * 1/2 CC : dC."""
    F = _F(dim, seed)
    C = F.T @ F
    rng = np.random.default_rng(seed)
    dC = rng.standard_normal((dim, dim))
    dC = dC + dC.T
    def S_of_C(Cm):
        Fm = np.linalg.cholesky(Cm).T       # any F with F^T F = C
        return M.pk2(Fm, np.float64(MU), np.float64(LAM))
    h = 1e-6
    fd = (S_of_C(C + h * dC) - S_of_C(C - h * dC)) / (2 * h)
    CC = M.referential_tangent(F, np.float64(MU), np.float64(LAM))
    np.testing.assert_allclose(0.5 * np.einsum("IJKL,KL->IJ", CC, dC), fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("dim,seed", [(2, 9), (3, 10)])
def test_push_forwards_match_printed_spatial_forms(dim, seed):
    F = _F(dim, seed)
    mu, lam = np.float64(MU), np.float64(LAM)
    tau = M.push_forward2(F, M.pk2(F, mu, lam))
    np.testing.assert_allclose(tau, M.tau_closed_form(F, mu, lam), atol=1e-12)
    jc = M.push_forward4(F, M.referential_tangent(F, mu, lam))
    np.testing.assert_allclose(jc, M.jc_closed_form(F, mu, lam), atol=1e-11)
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((dim, dim))
    G = G + G.T
    np.testing.assert_allclose(np.einsum("ijkl,kl->ij", jc, G), M.jc_action(F, mu, lam, G), atol=1e-11)


def test_undeformed_state_is_linear_elastic_with_mu_2lambda():
    """At F = I: S = 0 and CC = 2 mu Ssym + 2 lambda I(x)I (Lame pair (mu, 2 lambda))."""
    dim = 3
    F = np.eye(dim)
    np.testing.assert_allclose(M.pk2(F, np.float64(MU), np.float64(LAM)), 0.0, atol=1e-15)
    CC = M.referential_tangent(F, np.float64(MU), np.float64(LAM))
    eye = np.eye(dim)
    want = MU * (np.einsum("ik,jl->ijkl", eye, eye) + np.einsum("il,jk->ijkl", eye, eye)) \
        + 2 * LAM * np.einsum("ij,kl->ijkl", eye, eye)
    np.testing.assert_allclose(CC, want, atol=1e-14)


def test_objectivity_of_pk1():
    """P(QF) = Q P(F) for a rotation Q."""
    F = _F(3, 11)
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    mu, lam = np.float64(MU), np.float64(LAM)
    np.testing.assert_allclose(M.pk1(Q @ F, mu, lam), Q @ M.pk1(F, mu, lam), atol=1e-12)


# --- Mooney-Rivlin law (second law of the tensor4 route) ---

MU2 = 0.45


@pytest.mark.parametrize("dim,seed", [(2, 20), (2, 21), (3, 22), (3, 23)])
def test_mr_pk1_is_derivative_of_energy(dim, seed):
    F = _F(dim, seed)
    P = M.pk1(F, np.float64(MU), np.float64(LAM), np.float64(MU2))
    fd = _fd(lambda G: M.psi(G, MU, LAM, MU2), F)
    np.testing.assert_allclose(P, fd, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("dim,seed", [(2, 24), (3, 25), (3, 26)])
def test_mr_tangent_is_derivative_of_pk1(dim, seed):
    F = _F(dim, seed)
    A = M.dP_dF(F, np.float64(MU), np.float64(LAM), np.float64(MU2))
    fd = _fd(lambda G: M.pk1(G, np.float64(MU), np.float64(LAM), np.float64(MU2)), F)
    np.testing.assert_allclose(A, fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("dim,seed", [(2, 27), (3, 28)])
def test_mr_referential_tangent_is_second_derivative(dim, seed):
    F = _F(dim, seed)
    C = F.T @ F
    rng = np.random.default_rng(seed)
    dC = rng.standard_normal((dim, dim))
    dC = dC + dC.T
    def S_of_C(Cm):
        return M.pk2(np.linalg.cholesky(Cm).T, np.float64(MU), np.float64(LAM), np.float64(MU2))
    h = 1e-6
    fd = (S_of_C(C + h * dC) - S_of_C(C - h * dC)) / (2 * h)
    CC = M.referential_tangent(F, np.float64(MU), np.float64(LAM), np.float64(MU2))
    np.testing.assert_allclose(0.5 * np.einsum("IJKL,KL->IJ", CC, dC), fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("dim,seed", [(2, 29), (3, 30)])
def test_mr_push_forwards_match_spatial_closed_forms(dim, seed):
    """tau = chi(S) and J*c = chi(CC) (Sec. 2.1) against the spatial forms
    derived for the law; J*c keeps the minor and major symmetries."""
    F = _F(dim, seed)
    mu, lam, mu2 = np.float64(MU), np.float64(LAM), np.float64(MU2)
    tau = M.push_forward2(F, M.pk2(F, mu, lam, mu2))
    np.testing.assert_allclose(tau, M.mr_tau_closed_form(F, mu, lam, mu2), atol=1e-12)
    jc = M.push_forward4(F, M.referential_tangent(F, mu, lam, mu2))
    np.testing.assert_allclose(jc, M.mr_jc_closed_form(F, mu, lam, mu2), atol=1e-11)
    np.testing.assert_allclose(jc, jc.transpose(1, 0, 2, 3), atol=1e-12)
    np.testing.assert_allclose(jc, jc.transpose(2, 3, 0, 1), atol=1e-12)


def test_mr_with_zero_mu2_is_neo_hooke():
    F = _F(3, 31)
    mu, lam = np.float64(MU), np.float64(LAM)
    for f in (M.psi, M.pk2, M.referential_tangent, M.dP_dF):
        np.testing.assert_array_equal(f(F, mu, lam, 0.0), f(F, mu, lam))
    np.testing.assert_allclose(M.mr_tau_closed_form(F, mu, lam, 0.0), M.tau_closed_form(F, mu, lam), atol=1e-13)
    np.testing.assert_allclose(M.mr_jc_closed_form(F, mu, lam, 0.0), M.jc_closed_form(F, mu, lam), atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_mr_undeformed_state_is_linear_elastic(dim):
    """At F = I: psi = 0, S = 0, and CC is isotropic linear elasticity with
    Lame pair (mu + mu2, 2 lambda + 2 mu2) (plane strain for dim = 2)."""
    F = np.eye(dim)
    mu, lam, mu2 = np.float64(MU), np.float64(LAM), np.float64(MU2)
    assert abs(M.psi(F, mu, lam, mu2)) <= 1e-15
    np.testing.assert_allclose(M.pk2(F, mu, lam, mu2), 0.0, atol=1e-15)
    eye = np.eye(dim)
    want = (MU + MU2) * (np.einsum("ik,jl->ijkl", eye, eye) + np.einsum("il,jk->ijkl", eye, eye)) \
        + (2 * LAM + 2 * MU2) * np.einsum("ij,kl->ijkl", eye, eye)
    np.testing.assert_allclose(M.referential_tangent(F, mu, lam, mu2), want, atol=1e-14)


def test_mr_objectivity_and_uniaxial_closed_form():
    """P(QF) = Q P(F); for F = diag(s, 1, 1) the axial Kirchhoff stress is
    mu (s^2 - 1) + 2 mu2 (s^2 - 1) + 2 lambda ln s (I1 b - b^2 - 2 = 2 s^2 - 2
    on the axis), the lateral one mu2 (s^2 - 1) + 2 lambda ln s (there
    I1 b - b^2 - 2 = s^2 - 1)."""
    F = _F(3, 32)
    th = 0.4
    Q = np.array([[1.0, 0, 0], [0, np.cos(th), -np.sin(th)], [0, np.sin(th), np.cos(th)]])
    mu, lam, mu2 = np.float64(MU), np.float64(LAM), np.float64(MU2)
    np.testing.assert_allclose(M.pk1(Q @ F, mu, lam, mu2), Q @ M.pk1(F, mu, lam, mu2), atol=1e-12)
    s = 1.3
    Fu = np.diag([s, 1.0, 1.0])
    tau = Fu @ M.pk2(Fu, mu, lam, mu2) @ Fu.T
    ax = MU * (s * s - 1) + 2 * MU2 * (s * s - 1) + 2 * LAM * np.log(s)
    lat = MU2 * (s * s - 1) + 2 * LAM * np.log(s)
    np.testing.assert_allclose(np.diag(tau), [ax, lat, lat], rtol=1e-13)
