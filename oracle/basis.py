"""1-D building blocks of the tensor-product Q_p element (oracle, test
infrastructure only).

Sec. 5 writes every shape function and every quadrature point of a
tensor-product cell as a product of 1-D factors.  The oracle therefore needs
only 1-D objects, all on the unit interval [0, 1]:

* ``gll_points(p)``  support points of the degree-p Lagrange basis.  The paper
  does not name the point family; Gauss-Lobatto-Legendre is taken (it equals
  the equispaced family for p <= 2).
* ``gauss_rule(q)``  the q-point Gauss-Legendre rule; the paper uses q = p+1
  (Tables 1 and 2).
* ``lagrange(nodes, x)`` values and first derivatives of the Lagrange
  polynomials through ``nodes`` at the points ``x``, written out from the
  product definition.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll_points(p):
    """Degree-p Gauss-Lobatto-Legendre points on [0, 1], ascending.

    On [-1, 1] they are the two end points and the p-1 roots of P_p', the
    derivative of the Legendre polynomial of degree p.
    """
    if p < 1:
        raise ValueError("degree must be >= 1")
    inner = np.array([], dtype=np.float64)
    if p >= 2:
        coef = np.zeros(p + 1)
        coef[p] = 1.0
        inner = np.sort(np.real(npleg.legroots(npleg.legder(coef))))
    x = np.concatenate(([-1.0], inner, [1.0]))
    return 0.5 * (x + 1.0)


def gauss_rule(q):
    """q-point Gauss-Legendre points and weights on [0, 1] (weights sum to 1)."""
    x, w = npleg.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange(nodes, x):
    """Lagrange polynomials through ``nodes`` and their derivatives at ``x``.

    Returns (V, D) with V[k, a] = phi_a(x_k) and D[k, a] = phi_a'(x_k), where
    phi_a(t) = prod_{b != a} (t - t_b) / (t_a - t_b) and the derivative is the
    product rule applied to that product.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.zeros((len(x), n))
    D = np.zeros((len(x), n))
    for k, t in enumerate(x):
        for a in range(n):
            val = 1.0
            for b in range(n):
                if b != a:
                    val *= (t - nodes[b]) / (nodes[a] - nodes[b])
            V[k, a] = val
            der = 0.0
            for m in range(n):
                if m == a:
                    continue
                term = 1.0 / (nodes[a] - nodes[m])
                for b in range(n):
                    if b != a and b != m:
                        term *= (t - nodes[b]) / (nodes[a] - nodes[b])
                der += term
            D[k, a] = der
    return V, D
