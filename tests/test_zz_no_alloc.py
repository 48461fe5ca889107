"""The allocation-free dense inverse (mfh_dense_inverse_static, for callers
that cannot allocate device memory) against the workspace entry point
(mfh_dense_inverse), through the C ABI: calls in a row on one GPU, each
with a smaller matrix than the one before (the static work arrays keep the
previous call's contents), indefinite ones (pivoted pass) and a positive
definite one (plain pass), plus the size limit."""
import ctypes

import numpy as np
import pytest
import torch

from tests.gpu_helpers import host, log_case, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def _sym(n, seed, definite=False):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    eigs = rng.uniform(0.5, 2.0, n)
    if definite:                           # the plain pass is kept
        return (q * eigs) @ q.T
    A = (q * (eigs * rng.choice([-1.0, 1.0], n))) @ q.T
    A[: n // 4, : n // 4] = 0.0            # zero leading block: the pivoted pass runs
    return A


def test_static_dense_inverse_matches_workspace_entry():
    from paper_1904_13131_amd import dense_inverse
    for n, seed, definite in ((1000, 1, False), (301, 2, False), (200, 3, True)):
        log_case("dense_inverse_static", n=n, definite=definite)
        A = torch.as_tensor(_sym(n, seed, definite), device="cuda")
        ref, neg_ref = dense_inverse(A)
        got, neg = dense_inverse(A, static=True)
        r, g = host(ref), host(got)
        assert neg == neg_ref
        # same kernels, same order of operations on the same data: bitwise equal
        assert np.array_equal(r, g)
        An = host(A)
        assert np.linalg.norm(An @ g - np.eye(n)) / np.sqrt(n) <= 1e-9


def test_static_dense_inverse_size_limit():
    from paper_1904_13131_amd import MfhError, lib
    log_case("dense_inverse_static_limit")
    neg = ctypes.c_int()
    a = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = lib().mfh_dense_inverse_static(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(a.data_ptr() + 8), 2049,
                                        None, ctypes.byref(neg))
    assert st == -1
    msg = lib().mfh_last_error(None).decode()
    assert "2048" in msg
    with pytest.raises(MfhError):
        from paper_1904_13131_amd.mfh import _check
        _check(st)
