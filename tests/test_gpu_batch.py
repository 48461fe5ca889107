"""GPU tests of the batched path (many independent problems of different
meshes, degrees and materials) and of the graph-captured V-cycle."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fe
from paper_1904_13131_amd import F32, F64, Batch, Problem
from tests.gpu_helpers import dev, host, log_case, rel_l2, requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]

SMALL_LEVELS = {2: 2, 4: 2, 6: 2}


def sdev(a, dtype=torch.float64):
    """Device copy, synchronised (the problems run on their own streams)."""
    t = dev(a, dtype)
    torch.cuda.synchronize()
    return t


def _problems(n, seed, **kw):
    descs = W.batch_of_cubes(n=n, seed=seed, sizes=(2, 4, 6), degrees=(1, 2, 3))
    mu, lam = W.two_phase_material()
    probs, fields = [], []
    for d in descs:
        incl, u, x = W.batch_fields(d, coords=fe.Mesh(3, d["n_cells"], d["degree"]).coords_1d())
        s = torch.cuda.Stream()
        P = Problem(3, d["n_cells"], d["degree"], n_levels=SMALL_LEVELS[d["n_cells"]], mu=tuple(mu), lam=tuple(lam),
                    inclusions=incl, dirichlet_mask=d["mask"], stream=s, **kw)
        probs.append(P)
        fields.append((d, incl, u, x))
    torch.cuda.synchronize()
    return probs, fields


@pytest.mark.parametrize("policy", [0, 2], ids=["R", "C2"])
def test_batch_vmult_matches_single_and_oracle(policy):
    log_case("batch_vmult", policy=policy)
    probs, fields = _problems(14, 61, qp_policy=policy)
    us = [dev(f[2]) for f in fields]
    B = Batch(probs)
    mj = B.set_deformation(us)
    torch.cuda.synchronize()
    assert all(m > 0 for m in mj)
    for dt, tdt, tol in ((F64, torch.float64, 1e-13), (F32, torch.float32, 2e-6)):
        xs = [dev(f[3], tdt) for f in fields]
        # three calls: new pointers, the same pointers again, then other outputs
        outs = [[torch.full_like(x, float("nan")) for x in xs] for _ in range(2)]
        for ys in (outs[0], outs[0], outs[1]):
            B.tangent_vmult(xs, ys)
            torch.cuda.synchronize()
            for P, x, y in zip(probs, xs, ys):
                ref = P.tangent_vmult(x)
                torch.cuda.synchronize()
                assert rel_l2(host(y), host(ref)) <= tol
    # two problems against the oracle
    for k in (0, 5):
        d, incl, u, x = fields[k]
        m = fe.Mesh(3, d["n_cells"], d["degree"])
        mu, lam = W.two_phase_material()
        K = fe.constrain_matrix(fe.tangent_matrix(m, fe.Material(mu, lam, incl), u), m.constrained(d["mask"]))
        xs = [dev(f[3]) for f in fields]
        ys = [torch.empty_like(v) for v in xs]
        B.tangent_vmult(xs, ys)
        torch.cuda.synchronize()
        assert rel_l2(host(ys[k]), K @ x) <= 1e-12


@pytest.mark.parametrize("graphs", [False, True], ids=["eager", "graphs"])
def test_batch_cg_solve(graphs):
    """The lockstep batched PCG solves every problem as its own solve does
    (same iteration counts up to one, same solutions), a zero right-hand side
    included; one solution is checked against the oracle's assembled tangent."""
    log_case("batch_cg", graphs=graphs)
    probs, fields = _problems(8, 62, vcycle_dtype=F32)
    us = [dev(f[2]) for f in fields]
    B = Batch(probs)
    B.set_deformation(us)
    bs = []
    for k, ((d, incl, u, x), P) in enumerate(zip(fields, probs)):
        m = fe.Mesh(3, d["n_cells"], d["degree"])
        b = np.zeros_like(x) if k == 3 else x.copy()
        b[m.constrained(d["mask"])] = 0.0
        bs.append(dev(b))
    for P in probs:
        P.enable_graphs(graphs)
    xs = [torch.empty_like(b) for b in bs]
    torch.cuda.synchronize()
    it, rel, ms = B.cg_solve(bs, xs, rtol=1e-8, max_it=300)
    assert all(r <= 1e-8 for r in rel)
    assert it[3] == 0 and rel[3] == 0.0 and not host(xs[3]).any()
    assert all(m_ >= 0 for m_ in ms)
    for k, P in enumerate(probs):
        x1, it1, rel1, _ = P.cg_solve(bs[k], rtol=1e-8, max_it=300)
        torch.cuda.synchronize()
        assert abs(it1 - it[k]) <= 1, k
        if k != 3:
            assert rel_l2(host(xs[k]), host(x1)) <= 1e-7, k
    d, incl, u, x = fields[0]
    m = fe.Mesh(3, d["n_cells"], d["degree"])
    mu, lam = W.two_phase_material()
    K = fe.constrain_matrix(fe.tangent_matrix(m, fe.Material(mu, lam, incl), u), m.constrained(d["mask"]))
    b0 = host(bs[0])
    assert np.linalg.norm(b0 - K @ host(xs[0])) <= 1.05e-8 * np.linalg.norm(b0)


@pytest.mark.parametrize("dim,n,p", [(3, 4, 3), (2, 6, 4), (3, 8, 1)])
def test_node_coords_match_oracle(dim, n, p):
    log_case("node_coords", dim=dim, n=n, p=p)
    P = Problem(dim, n, p, n_levels=2)
    for level in (0, 1):
        m = fe.Mesh(dim, n >> (1 - level), p)
        np.testing.assert_allclose(P.node_coords_1d(level), m.coords_1d(), rtol=0, atol=1e-15)


def test_batch_set_deformation_reports_inverted_problem():
    """One problem of the batch gets an inverting displacement: the batch
    reports INVERTED naming it, and the other problems stay usable."""
    from paper_1904_13131_amd import MfhError
    log_case("batch_inverted")
    probs, fields = _problems(3, 63)
    us = [dev(f[2]) for f in fields]
    m1 = fe.Mesh(3, fields[1][0]["n_cells"], fields[1][0]["degree"])
    X = m1.node_coords()
    bad = np.ascontiguousarray((-1.5 * X).T.reshape(-1))   # F = -0.5 I: det < 0 everywhere
    us[1] = dev(bad)
    B = Batch(probs)
    with pytest.raises(MfhError) as e:
        B.set_deformation(us)
    assert e.value.name == "INVERTED" and "problem 1" in str(e.value)
    x = dev(fields[0][3])
    y = probs[0].tangent_vmult(x)
    torch.cuda.synchronize()
    assert np.isfinite(host(y)).all()


@pytest.mark.parametrize("vdt", [F64, F32], ids=["f64", "f32"])
def test_graph_vcycle_replays_match_eager(vdt):
    """The captured V-cycle is replayed several times with eager work and
    synchronisations in between; every replay equals the eager V-cycle."""
    log_case("graph_replay", vcycle=vdt)
    mu, lam = W.two_phase_material()
    incl = W.spheres(3, 3)
    s = torch.cuda.Stream()
    P = Problem(3, 8, 2, n_levels=3, mu=tuple(mu), lam=tuple(lam), inclusions=incl,
                dirichlet_mask=W.clamp_bottom_top(3), vcycle_dtype=vdt, stream=s)
    m = fe.Mesh(3, 8, 2)
    cons = m.constrained(W.clamp_bottom_top(3))
    u = W.stretched_field(3, m.L, 0.05, 4, 0.0125)
    b = W.normal_vector(m.n_dofs, 8)
    b[cons] = 0.0
    torch.cuda.synchronize()
    P.set_deformation(sdev(u))
    z_eager = host(P.gmg_vcycle(sdev(b)))
    P.enable_graphs(True)
    tol = 1e-12 if vdt == F64 else 2e-5
    other = sdev(W.normal_vector(m.n_dofs, 9))
    for rep in range(4):
        z = host(P.gmg_vcycle(sdev(b)))
        assert rel_l2(z, z_eager) <= tol, rep
        P.tangent_vmult(other)            # eager work between replays
        torch.cuda.synchronize()
    x_g, it_g, rel_g, _ = P.cg_solve(sdev(b), rtol=1e-8, max_it=200)
    P.enable_graphs(False)
    x_e, it_e, rel_e, _ = P.cg_solve(sdev(b), rtol=1e-8, max_it=200)
    assert rel_g <= 1e-8 and rel_e <= 1e-8
    assert abs(it_g - it_e) <= 1
    assert rel_l2(host(x_g), host(x_e)) <= 1e-7


def _real_subset(k=8, seed=66):
    """A seeded subset of the 256-problem batch at its real sizes, covering
    every degree and every mesh size of the recipe."""
    descs = W.batch_of_cubes()
    rng = np.random.default_rng(seed)
    pick, seen = [], set()
    for i in rng.permutation(len(descs)):      # first cover each (degree, N) pair seen in order
        key = (descs[i]["degree"], descs[i]["n_cells"])
        if key not in seen:
            seen.add(key)
            pick.append(int(i))
        if len(pick) == k:
            break
    return [descs[i] for i in sorted(pick)]


def test_batch_real_sizes_against_oracle_rows():
    """Eight problems of the batch at their real sizes (8^3..24^3 cells, Q1..Q3,
    up to 1.17 M DoFs) in one batched vmult, FP64 and FP32, against the
    oracle's assembled tangent on sampled rows (corner, edge, face and
    interior nodes of every component)."""
    descs = _real_subset()
    assert {d["degree"] for d in descs} == {1, 2, 3} and len({d["n_cells"] for d in descs}) >= 3
    mu, lam = W.two_phase_material()
    probs, fields = [], []
    for d in descs:
        log_case("batch_real", n_cells=d["n_cells"], degree=d["degree"])
        m = fe.Mesh(3, d["n_cells"], d["degree"])
        incl, u, x = W.batch_fields(d, coords=m.coords_1d())
        P = Problem(3, d["n_cells"], d["degree"], n_levels=d["n_levels"], mu=tuple(mu), lam=tuple(lam),
                    inclusions=incl, dirichlet_mask=d["mask"], qp_policy=2, stream=torch.cuda.Stream())
        probs.append(P)
        fields.append((d, m, incl, u, x))
    torch.cuda.synchronize()
    B = Batch(probs)
    assert all(mj > 0 for mj in B.set_deformation([sdev(f[3]) for f in fields]))
    for dt, tdt in ((F64, torch.float64), (F32, torch.float32)):
        xs = [sdev(f[4], tdt) for f in fields]
        ys = [torch.full_like(x, float("nan")) for x in xs]
        B.tangent_vmult(xs, ys)
        torch.cuda.synchronize()
        for (d, m, incl, u, x), y in zip(fields, ys):
            L = m.L
            rng = np.random.default_rng(d["x_seed"])
            nodes = np.r_[0, L - 1, L * L - 1, m.n_nodes - 1, L * (L // 2) + L // 2,
                          rng.choice(m.n_nodes, 20, replace=False)]
            rows = np.unique(np.concatenate([nodes + c * m.n_nodes for c in range(3)]))
            xin = x if dt == F64 else x.astype(np.float32).astype(np.float64)
            ref = fe.vmult_rows(m, fe.Material(mu, lam, incl), u, xin, rows, m.constrained(d["mask"]))
            got = host(y)[rows]
            err = np.abs(got - ref).max() / np.abs(ref).max()
            print(f"[batch_real] N {d['n_cells']} p {d['degree']} {'f64' if dt == F64 else 'f32'}: "
                  f"max rel {err:.2e}", flush=True)
            assert err <= (1e-12 if dt == F64 else 1e-5)
            assert np.all(np.isfinite(host(y)))


@pytest.mark.parametrize("policy", [0, 2, 3], ids=["R", "C2", "C4"])
def test_batch_fused_launch_matches_per_degree(policy):
    """The persistent launch over every degree computes what the per-degree
    launches compute (same block bodies; the atomic-scatter problems differ
    only by summation order), FP64 and FP32, and a 2-D batch refuses it."""
    from paper_1904_13131_amd import MfhError
    from paper_1904_13131_amd.mfh import BATCH_LAUNCH_AUTO, BATCH_LAUNCH_FUSED, BATCH_LAUNCH_PER_DEGREE
    log_case("batch_fused", policy=policy)
    probs, fields = _problems(12, 63, qp_policy=policy)
    B = Batch(probs)
    B.set_deformation([dev(f[2]) for f in fields])
    for tdt, tol in ((torch.float64, 1e-13), (torch.float32, 2e-6)):
        xs = [dev(f[3], tdt) for f in fields]
        outs = {}
        for mode in (BATCH_LAUNCH_PER_DEGREE, BATCH_LAUNCH_FUSED, BATCH_LAUNCH_AUTO):
            ys = [torch.full_like(x, float("nan")) for x in xs]
            B.set_launch(mode)
            B.tangent_vmult(xs, ys)
            torch.cuda.synchronize()
            outs[mode] = [host(y) for y in ys]
        for a, b, c in zip(outs[BATCH_LAUNCH_PER_DEGREE], outs[BATCH_LAUNCH_FUSED], outs[BATCH_LAUNCH_AUTO]):
            assert np.all(np.isfinite(b))
            assert rel_l2(b, a) <= tol and rel_l2(c, a) <= tol
    P2 = Problem(2, 4, 2, mu=(1.0,), lam=(1.5,))
    B2 = Batch([P2])
    with pytest.raises(MfhError):
        B2.set_launch(BATCH_LAUNCH_FUSED)
