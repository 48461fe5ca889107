"""End-to-end pin of the oracle Newton + GMG-CG (Sec. 3, Sec. 6, Sec. 7):
uniaxial stretch of a homogeneous cube on rollers has the affine exact
solution F = diag(s, s, 1 + delta) with mu s^2 = mu - 2 lambda ln(s^2 (1 + delta))
(lateral Kirchhoff stress tau = mu b - c1 I vanishes), which lies in the
finite-element space, so the discrete solution equals it."""
import numpy as np
import pytest
from scipy.optimize import brentq

import workloads as W
from oracle import fe, gmg, newton


@pytest.mark.parametrize("dim,p,delta", [(3, 2, 0.1), (2, 3, -0.15), (3, 1, 0.08)])
def test_uniaxial_stretch_closed_form(dim, p, delta):
    mu, lam = 1.0, 1.5
    mat = fe.Material([mu], [lam])
    ax = dim - 1
    mask = W.face_bits(dim, ax, 0, [ax]) | W.face_bits(dim, ax, 1, [ax])
    for a in range(dim - 1):
        mask |= W.face_bits(dim, a, 0, [a])
    vals = np.zeros((2 * dim, dim))
    vals[2 * ax + 1][ax] = delta
    H = gmg.Hierarchy(dim, 1, p, 2, mat, mask)
    u, recs = newton.solve(H, vals, n_steps=2)
    s = brentq(lambda s: mu * s * s - (mu - 2 * lam * np.log(s ** (dim - 1) * (1 + delta))), 0.5, 1.5)
    m = H.meshes[-1]
    X = m.node_coords()
    want = X * np.array([s - 1] * (dim - 1) + [delta])
    np.testing.assert_allclose(u.reshape(dim, -1).T, want, atol=1e-9)
    # reaction on the moving face: sum of unconstrained residual = P_zz * area
    R = fe.residual(m, mat, u).reshape(dim, -1).T
    top = np.abs(X[:, ax] - 1.0) < 1e-12
    Pzz = (mu * (1 + delta) ** 2 - (mu - 2 * lam * np.log(s ** (dim - 1) * (1 + delta)))) / (1 + delta)
    assert abs(R[top, ax].sum() - Pzz) < 1e-9
    assert all(r["cg_rel"] <= 1e-8 for r in recs)


def test_cutback_reaches_the_same_equilibrium():
    """A stiff disc compressed 30 % in one increment: the first Newton
    iterates hit negative curvature (CG breakdown), so the driver halves the
    failed increment; the converged state is the one four uncut increments
    reach (the equilibrium of a hyperelastic body does not depend on the
    loading path while it stays on one branch)."""
    mu, lam = W.two_phase_material()
    mat = fe.Material(mu, lam, [(np.array([0.5, 0.5]), 0.3, 1)])
    H = gmg.Hierarchy(2, 2, 2, 3, mat, W.clamp_bottom_top(2))
    fv = np.zeros((4, 2))
    fv[3][1] = -0.3
    u1, r1 = newton.solve(H, fv, n_steps=1)
    u4, r4 = newton.solve(H, fv, n_steps=4)
    assert max(r["cutbacks"] for r in r1) == 2 and max(r["cutbacks"] for r in r4) == 0
    assert [r["load_fraction"] for r in r1 if not np.isfinite(r["cg_rel"])] == [1.0, 1.0]
    assert r1[-1]["load_fraction"] == 1.0
    assert np.linalg.norm(u1 - u4) <= 1e-10 * np.linalg.norm(u4)


def test_shortened_step_reaches_the_same_equilibrium():
    """The same body compressed 35 % in one increment: the full first step
    inverts a quadrature point, so the step length halves (alpha = 1/2) and
    the next step carries the rest of the prescribed values; after cut-backs
    the converged state is the one seven uncut increments reach.  A wrong
    remainder of the prescribed values would leave the top face short of
    -0.35; a shortened step that skipped the J > 0 test would stop at NaN."""
    mu, lam = W.two_phase_material()
    mat = fe.Material(mu, lam, [(np.array([0.5, 0.5]), 0.3, 1)])
    H = gmg.Hierarchy(2, 2, 2, 3, mat, W.clamp_bottom_top(2))
    fv = np.zeros((4, 2))
    fv[3][1] = -0.35
    u1, r1 = newton.solve(H, fv, n_steps=1)
    u7, r7 = newton.solve(H, fv, n_steps=7)
    assert r1[0]["alpha"] == 0.5 and np.isfinite(r1[0]["res_after"])
    assert all(r["alpha"] == 1.0 for r in r7)
    assert r1[-1]["load_fraction"] == 1.0
    top = H.meshes[-1].n_nodes + np.arange(H.meshes[-1].L ** 2 - H.meshes[-1].L, H.meshes[-1].L ** 2)
    assert np.all(u1[top] == -0.35)
    assert np.linalg.norm(u1 - u7) <= 1e-10 * np.linalg.norm(u7)


@pytest.mark.parametrize("dim,p", [(3, 2), (2, 3), (3, 1)])
def test_external_force_totals(dim, p):
    """The nodal forces of a constant traction on a unit face sum to the
    traction (times the face area 1) per component, vanish off the face, and
    reproduce the face integral of a linear field (first moments)."""
    m = fe.Mesh(dim, 3, p)
    ft = np.zeros((2 * dim, dim))
    ft[2 * (dim - 1) + 1] = np.arange(1, dim + 1)        # top face
    f = fe.external_force(m, ft)
    X = m.node_coords()
    top = np.abs(X[:, dim - 1] - 1.0) < 1e-12
    for c in range(dim):
        fc = f[c * m.n_nodes:(c + 1) * m.n_nodes]
        assert abs(fc.sum() - (c + 1)) < 1e-13
        assert np.all(fc[~top] == 0)
        # sum_a f_a X_a = t * integral of X over the face = t * 1/2 (first tangential axis)
        assert abs((fc * X[:, 0]).sum() - 0.5 * (c + 1)) < 1e-13


def test_uniaxial_traction_closed_form():
    """Traction control: a dead traction t on the top face of a cube on
    rollers gives the homogeneous state F = diag(s, s, 1 + delta) with zero
    lateral stress and first Piola stress P_zz = t; the state is affine, so
    the discrete solution equals it."""
    dim, mu, lam, t = 3, 1.0, 1.5, 0.08
    mat = fe.Material([mu], [lam])
    mask = W.face_bits(dim, 2, 0, [2]) | W.face_bits(dim, 0, 0, [0]) | W.face_bits(dim, 1, 0, [1])
    H = gmg.Hierarchy(dim, 1, 2, 2, mat, mask)
    ft = np.zeros((6, 3))
    ft[5][2] = t
    u, recs = newton.solve(H, np.zeros((6, 3)), n_steps=2, face_traction=ft)
    # lateral: mu s^2 = c1, axial: P_zz = (mu (1+d)^2 - c1) / (1+d) = t, c1 = mu - 2 lam ln(s^2 (1+d))
    def eqs(v):
        s, d = v
        c1 = mu - 2 * lam * np.log(s * s * (1 + d))
        return [mu * s * s - c1, (mu * (1 + d) ** 2 - c1) / (1 + d) - t]
    from scipy.optimize import fsolve
    s, d = fsolve(eqs, [1.0, 0.05], xtol=1e-14)
    X = H.meshes[-1].node_coords()
    want = X * np.array([s - 1, s - 1, d])
    np.testing.assert_allclose(u.reshape(dim, -1).T, want, atol=1e-9)
