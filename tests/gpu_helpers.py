"""Shared helpers of the GPU parity tests: build a device problem and the
matching oracle objects from one synthetic workload dict."""
import numpy as np
import pytest
import torch

from oracle import fe

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def device_problem(w, n_levels=1, **kw):
    from paper_1904_13131_amd import Problem
    return Problem(w["dim"], w["n_cells"], w["degree"], n_levels=n_levels,
                   mu=tuple(w["mu"]), lam=tuple(w["lam"]), inclusions=w["inclusions"],
                   dirichlet_mask=w["mask"], **kw)


def oracle_problem(w):
    mesh = fe.Mesh(w["dim"], w["n_cells"], w["degree"])
    mat = fe.Material(w["mu"], w["lam"], w["inclusions"])
    cons = mesh.constrained(w["mask"])
    return mesh, mat, cons


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel_max(a, b):
    """Largest entry error against the largest reference entry."""
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def log_case(_case, **kw):
    print(f"[case] {_case} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
