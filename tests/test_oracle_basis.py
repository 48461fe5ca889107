"""Pins for the oracle's 1-D building blocks (Sec. 5 tensor-product bases,
q = p+1 Gauss rule of Tables 1-2)."""
import math
import os

import numpy as np
import pytest

from oracle import basis, fe

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "quadrature_1d.txt")


def _golden():
    rows = []
    env = {"sqrt": math.sqrt, "__builtins__": {}}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        tok = line.split()
        kind, n = tok[0], int(tok[1])
        xs = [eval(t, env) for t in tok[2:2 + n]]
        ws = None if tok[2 + n] == "-" else [eval(t, env) for t in tok[2 + n:2 + 2 * n]]
        rows.append((kind, n, np.array(xs), None if ws is None else np.array(ws)))
    return rows


@pytest.mark.parametrize("row", _golden(), ids=lambda r: f"{r[0]}{r[1]}")
def test_points_match_tables(row):
    kind, n, xs, ws = row
    if kind == "gauss":
        x, w = basis.gauss_rule(n)
        np.testing.assert_allclose(x, 0.5 * (xs + 1), atol=1e-14)
        np.testing.assert_allclose(w, 0.5 * ws, atol=1e-14)
    else:
        np.testing.assert_allclose(basis.gll_points(n - 1), 0.5 * (xs + 1), atol=1e-14)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5, 6])
def test_gauss_exact_to_degree_2q_minus_1(q):
    x, w = basis.gauss_rule(q)
    for k in range(2 * q):
        assert abs(w @ x ** k - 1.0 / (k + 1)) < 1e-14
    # and not beyond: degree 2q is integrated with an error
    assert abs(w @ x ** (2 * q) - 1.0 / (2 * q + 1)) > 1e-9


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lagrange_delta_and_partition(p):
    xi = basis.gll_points(p)
    V, D = basis.lagrange(xi, xi)
    np.testing.assert_allclose(V, np.eye(p + 1), atol=1e-13)
    t = np.linspace(0, 1, 17)
    V, D = basis.lagrange(xi, t)
    np.testing.assert_allclose(V.sum(axis=1), 1.0, atol=1e-13)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-11)
    # reproduces every polynomial of degree <= p with its derivative
    for k in range(p + 1):
        np.testing.assert_allclose(V @ xi ** k, t ** k, atol=1e-12)
        np.testing.assert_allclose(D @ xi ** k, k * t ** max(k - 1, 0) if k else 0 * t, atol=1e-10)


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 3), (3, 2), (3, 4)])
def test_reference_gradients_reproduce_polynomials(dim, p):
    """sum_a f(X_a) G[q, a, :] = grad f(X_q) for f of degree <= p per axis."""
    m = fe.Mesh(dim, 3, p)
    rng = np.random.default_rng(0)
    c = rng.standard_normal((p + 1,) * dim)
    def f(X):
        val = np.zeros(X.shape[0])
        grad = np.zeros_like(X)
        for idx in np.ndindex(*c.shape):
            mono = np.prod([X[:, k] ** idx[k] for k in range(dim)], axis=0)
            val += c[idx] * mono
            for I in range(dim):
                if idx[I]:
                    g = idx[I] * np.prod([X[:, k] ** (idx[k] - (k == I)) for k in range(dim)], axis=0)
                    grad[:, I] += c[idx] * g
        return val, grad
    X = m.node_coords()
    fv, _ = f(X)
    cells = np.array([0, m.n_cells - 1, m.n_cells // 2])
    nodes = m.cell_nodes(cells)
    got = np.einsum("ca,qaI->cqI", fv[nodes], m.G)
    _, want = f(m.qp_coords(cells).reshape(-1, dim))
    np.testing.assert_allclose(got.reshape(-1, dim), want, atol=1e-9)
    np.testing.assert_allclose(m.W.sum() * m.n_cells, 1.0, atol=1e-14)
