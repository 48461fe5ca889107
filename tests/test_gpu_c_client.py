"""The C ABI from a plain C program (tests/c_client.c: hipMalloc'd buffers,
mfh_create, mfh_set_deformation, mfh_tangent_vmult, mfh_cg_solve) on a 3-D Q2
body with a stiff sphere, clamped at the bottom and top: K_c x against the
oracle's assembled constrained tangent (1e-12), and the CG solution's true
residual with the oracle's matrix (1e-8, the requested tolerance)."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import fe
from tests.c_client_build import build_client
from tests.gpu_helpers import log_case, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def test_c_client_vmult_and_cg(tmp_path):
    n = 8
    log_case("c_client", n_cells=n)
    mask = W.clamp_bottom_top(3)
    mesh = fe.Mesh(3, n, 2)
    mat = fe.Material([1.0, 100.0], [1.5, 150.0], [((0.5, 0.5, 0.5), 0.2, 1)])
    cons = mesh.constrained(mask)
    u = W.sine_field(3, mesh.L, 4, 0.05, kmax=1)
    u[cons] = 0.0
    x = W.normal_vector(mesh.n_dofs, 5)
    x[cons] = 0.0
    for name, v in (("u", u), ("x", x)):
        v.astype(np.float64).tofile(str(tmp_path / f"{name}.bin"))
    exe = build_client(str(tmp_path))
    r = subprocess.run([exe, str(n), str(tmp_path / "u.bin"), str(tmp_path / "x.bin"), str(tmp_path / "y.bin"),
                        str(tmp_path / "z.bin")], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0
    y = np.fromfile(str(tmp_path / "y.bin"), dtype=np.float64)
    z = np.fromfile(str(tmp_path / "z.bin"), dtype=np.float64)
    K = fe.constrain_matrix(fe.tangent_matrix(mesh, mat, u), cons).tocsc()
    yo = K @ x
    assert np.linalg.norm(y - yo) <= 1e-12 * np.linalg.norm(yo)
    assert np.linalg.norm(x - K @ z) <= 1.05e-8 * np.linalg.norm(x)
    fields = dict(zip(r.stdout.split()[0::2], r.stdout.split()[1::2]))
    assert int(fields["n_dofs"]) == mesh.n_dofs and float(fields["relres"]) <= 1e-8
