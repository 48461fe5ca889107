"""CPU checks of the C ABI: the library loads, exports every function the
header declares, validates descriptors on the host, and the product package
never touches the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfh.h")
LIB = os.path.join(ROOT, "paper_1904_13131_amd", "libmfh.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfh_[a-z_0-9]+)\s*\(", text)))


def _lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built: run python -m paper_1904_13131_amd.build")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["mfh_workspace_size", "mfh_create", "mfh_destroy", "mfh_set_deformation", "mfh_tangent_vmult",
                 "mfh_residual", "mfh_gmg_vcycle", "mfh_cg_solve", "mfh_last_error", "mfh_newton_solve"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def _desc(**kw):
    from paper_1904_13131_amd import make_desc
    base = dict(dim=3, n_cells=8, degree=2, n_levels=2, mu=(1.0, 100.0), lam=(1.5, 150.0))
    base.update(kw)
    return make_desc(**base)


def test_workspace_size_on_host():
    from paper_1904_13131_amd import workspace_size
    d, keep = _desc()
    n1 = workspace_size(d)
    d2, keep2 = _desc(n_cells=16, n_levels=3)
    assert workspace_size(d2) > n1 > 0


@pytest.mark.parametrize("bad", [
    dict(dim=4), dict(degree=0), dict(degree=5), dict(n_cells=0), dict(n_cells=1024, degree=2, n_levels=1), dict(n_cells=6, n_levels=3),
    dict(mu=(-1.0,), lam=(1.0,)), dict(qp_policy=4), dict(qp_policy=-1), dict(scatter=4), dict(scatter=-2), dict(vcycle_dtype=5),
    dict(cheb_degree=0), dict(n_smooth=0), dict(eig_iters=0), dict(cheb_lo=1.3, cheb_hi=1.2),
    dict(dirichlet_mask=1 << 18), dict(level_field=2), dict(coarse_solver=2), dict(eig_refresh=-1), dict(inclusions=[((0.5, 0.5, 0.5), 0.2, 2)]),
    dict(law=2), dict(law=1, qp_policy=2, mu2=(0.3, 30.0)), dict(law=1, qp_policy=3, mu2=(-0.3, 30.0)),
    dict(law=1, qp_policy=3, mu2=(float("nan"), 30.0)), dict(tile_shape=2), dict(tile_shape=-2), dict(cell_block=2), dict(cell_block=-2),
])
def test_invalid_descriptors_rejected(bad):
    from paper_1904_13131_amd import MfhError, workspace_size
    d, keep = _desc(**bad)
    with pytest.raises(MfhError) as e:
        workspace_size(d)
    assert e.value.name == "INVALID_ARG"


def test_tensor4_and_second_law_accepted():
    """CACHE_T4 with either law; its cache is 36 words per quadrature point in
    3-D (F^-1, S, J c), so the workspace grows over CACHE_T2's 10 (F^-1, c1)."""
    from paper_1904_13131_amd import workspace_size
    sizes = {}
    for pol, law in ((2, 0), (3, 0), (3, 1)):
        d, keep = _desc(qp_policy=pol, law=law, mu2=(0.3, 30.0))
        sizes[(pol, law)] = workspace_size(d)
    assert sizes[(3, 0)] == sizes[(3, 1)] > sizes[(2, 0)]
    n_cells, nq = 8 ** 3, 27
    d2, keep2 = _desc(n_levels=1, qp_policy=2)
    d3, keep3 = _desc(n_levels=1, qp_policy=3)
    assert workspace_size(d3) - workspace_size(d2) == (36 - 10) * nq * n_cells * 12   # FP64 + FP32 copies


def test_create_rejects_small_or_null_workspace():
    from paper_1904_13131_amd import make_desc, mfh
    L = mfh.lib()
    d, keep = make_desc(2, 4, 1)
    h = ctypes.c_void_p()
    st = L.mfh_create(ctypes.byref(d), None, 0, None, ctypes.byref(h))
    assert st == -1
    assert b"workspace" in L.mfh_last_error(None)


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1904_13131_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.replace("oracle_", ""), f


# --- argument checks of the binding (host only: every case is refused before
# any pointer reaches the library, so no kernel is launched) ---

def _fake_problem(n=81, levels=2):
    import torch
    from paper_1904_13131_amd import mfh
    P = mfh.Problem.__new__(mfh.Problem)
    P.desc, P._keep = _desc(n_levels=levels)
    P.device = torch.device("cuda", 0)
    P.dim, P.n_levels, P.handle = 3, levels, None
    P.n_dofs = lambda level=-1: n if level % levels == levels - 1 else n // 3
    return P


def test_binding_rejects_bad_vectors():
    import torch
    P = _fake_problem()
    cpu = torch.zeros(81, dtype=torch.float64)
    with pytest.raises(ValueError, match="device"):
        P.tangent_vmult(cpu)
    with pytest.raises(ValueError, match="device"):
        P.set_deformation(cpu)
    with pytest.raises(ValueError, match="device"):
        P.residual(cpu)
    with pytest.raises(ValueError, match="device"):
        P.cg_solve(cpu)
    with pytest.raises(ValueError, match="device"):
        P.gmg_vcycle(cpu)
    with pytest.raises(ValueError, match="tensor"):
        P.tangent_vmult([0.0] * 81)


def test_binding_checks_dtype_size_and_layout():
    import torch
    from paper_1904_13131_amd import mfh
    dev = torch.device("cuda", 0)
    meta = lambda n, dt=torch.float64: torch.empty(n, dtype=dt, device="meta")
    # _arg itself, on tensors that never hold device memory
    with pytest.raises(ValueError, match="device"):
        mfh._arg(meta(81), "x", dev, 81)
    x = torch.zeros(81, dtype=torch.float64)
    cpu = torch.device("cpu")
    mfh._arg(x, "x", cpu, 81)
    with pytest.raises(ValueError, match="entries"):
        mfh._arg(x, "x", cpu, 80)
    with pytest.raises(ValueError, match="dtype"):
        mfh._arg(x.float(), "x", cpu, 81)
    with pytest.raises(ValueError, match="contiguous"):
        mfh._arg(torch.zeros(162, dtype=torch.float64)[::2], "x", cpu, 81)
    with pytest.raises(ValueError, match="dtype"):
        mfh._arg(x, "x", cpu, 81, (torch.float32,))


def test_binding_checks_levels_faces_and_batches():
    import torch
    from paper_1904_13131_amd import mfh
    P = _fake_problem()
    P.device = torch.device("cpu")              # lets the checks reach the level and face tests
    x = torch.zeros(27, dtype=torch.float64)
    with pytest.raises(ValueError, match="level"):
        P.prolongate(0, x)
    with pytest.raises(ValueError, match="level"):
        P.restrict(2, x)
    with pytest.raises(ValueError, match="entries"):
        P.prolongate(1, torch.zeros(81, dtype=torch.float64))
    with pytest.raises(ValueError, match="faces"):
        P.apply_dirichlet(torch.zeros(81, dtype=torch.float64), [[0.0, 0.0, 0.0]] * 5)
    with pytest.raises(ValueError, match="dtype"):        # output dtype must follow the input
        P.tangent_vmult(torch.zeros(81, dtype=torch.float64), torch.zeros(81, dtype=torch.float32))
    B = mfh.Batch.__new__(mfh.Batch)
    B.problems, B.handle = [P, P], None
    ok = torch.zeros(81, dtype=torch.float64)
    with pytest.raises(ValueError, match="problems"):
        B.tangent_vmult([ok], [ok])
    with pytest.raises(ValueError, match="problems"):
        B.set_deformation([ok, ok, ok])
    with pytest.raises(ValueError, match="mixed"):
        B.tangent_vmult([ok, ok.float()], [ok, ok])
    with pytest.raises(ValueError, match="dtype"):
        B.tangent_vmult([ok, ok], [ok.float(), ok.float()])
    with pytest.raises(ValueError, match="entries"):
        B.cg_solve([ok, ok], [ok, torch.zeros(80, dtype=torch.float64)])


def test_c_client_compiles_and_links(tmp_path):
    """include/mfh.h is plain C: a C99 client (tests/c_client.c) compiles with
    -Wall -Wextra -Werror and links against the library and the HIP runtime
    alone (no Python, no torch)."""
    from tests.c_client_build import build_client
    _lib()
    exe = build_client(str(tmp_path))
    assert os.path.exists(exe)
