"""GPU tests of the coarse level's dense direct solver (the exact FP64 coarse
solve of the V-cycle) on matrices with known inverses and inertia: the plain
pass where it is accurate, symmetric pivoting where it is not (zero or small
leading minors, saddle-point matrices); the negative pivot count equals the
number of negative eigenvalues (Sylvester's law of inertia); singular
matrices are reported."""
import numpy as np
import pytest
import torch

from tests.gpu_helpers import host, log_case, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]
EPS = np.finfo(np.float64).eps


def _sym(n, seed, eigs=None):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    if eigs is None:
        eigs = rng.uniform(0.5, 2.0, n) * rng.choice([-1.0, 1.0], n)
    return (q * eigs) @ q.T


def _saddle(n, k, seed):
    """[[0, B^T], [B, C]] with a k x k zero block: every leading principal
    minor of order <= k vanishes; nonsingular (B full column rank, C SPD),
    with exactly k negative eigenvalues."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n - k, k))
    C = _sym(n - k, seed + 1, rng.uniform(1.0, 3.0, n - k))
    A = np.zeros((n, n))
    A[k:, :k] = B
    A[:k, k:] = B.T
    A[k:, k:] = C
    return A


CASES = {
    "swap_2": np.array([[0.0, 1.0], [1.0, 0.0]]),
    "one": np.array([[-3.0]]),
    "saddle_200_zero_block_70": _saddle(200, 70, 3),
    "saddle_131_zero_block_64": _saddle(131, 64, 4),
    "indefinite_300": _sym(300, 5),
    "spd_197": _sym(197, 6, np.geomspace(1e-2, 1e2, 197)),
    "tiny_first_pivot_150": None,
}
A = _sym(150, 7)
A[0, 0] = 1e-14                      # a leading 1x1 minor that is not zero, only tiny
CASES["tiny_first_pivot_150"] = A
A = _sym(150, 7)
A[0, 0] = 1e-9                       # above the singularity threshold: the plain pass
CASES["small_first_pivot_150"] = A   # grows entries ~1e9 and must be rejected


@pytest.mark.parametrize("name", list(CASES))
def test_dense_inverse(name):
    from paper_1904_13131_amd import dense_inverse
    log_case("dense_inverse", name=name)
    A = CASES[name]
    n = A.shape[0]
    inv, neg = dense_inverse(torch.as_tensor(A, device="cuda"))
    X = host(inv)
    ev = np.linalg.eigvalsh(A)
    assert neg == int((ev < 0).sum())
    kappa = np.abs(ev).max() / np.abs(ev).min()
    res = np.linalg.norm(A @ X - np.eye(n)) / np.sqrt(n)
    print(f"[dense_inverse] {name}: n {n}, kappa {kappa:.1e}, |AX - I| {res:.2e}, negative {neg}", flush=True)
    # Gauss-Jordan with bounded element growth: residual of order n u kappa
    assert res <= 10 * n * EPS * kappa
    np.testing.assert_allclose(X, X.T, atol=10 * n * EPS * kappa * np.abs(X).max())


def test_dense_inverse_rejects_singular():
    from paper_1904_13131_amd import MfhError, dense_inverse
    log_case("dense_inverse_singular")
    w = np.random.default_rng(10).standard_normal(90)
    w /= np.linalg.norm(w)
    P = np.eye(90) - np.outer(w, w)
    A = P @ _sym(90, 9) @ P          # symmetric with A w = 0
    with pytest.raises(MfhError) as e:
        dense_inverse(torch.as_tensor(A, device="cuda"))
    assert e.value.name == "NOT_SPD"
