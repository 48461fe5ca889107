"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only draws random numbers
and writes them into plain arrays (sphere lists, nodal displacement values,
right-hand sides).  Both the device path and the oracle consume its output.

Recipes
-------
* Material: matrix mu = 1, nu = 0.3 -> lambda = 2 mu nu / (1 - 2 nu) = 1.5;
  inclusions are 100x stiffer in both parameters (mu = 100, lambda = 150).
* Spheres: for each of n spheres, r ~ U[rmin, rmax], then the centre
  ~ U[r, 1 - r]^d, drawn in that order from ``numpy.random.default_rng(seed)``.
* Displacement: u_c(X) = s * sum_m a_mc sin(pi k_m . X + phi_m) with
  a_m ~ N(0, 1)^d, k_m drawn uniformly from {0..kmax}^d minus the zero vector,
  phi_m ~ U[0, 2 pi); X is the node position when the caller passes the
  support-point coordinates along an axis (``coords``), else the lattice
  parameter index / (L - 1) (the same for degrees 1 and 2, whose support
  points are equispaced; for higher degrees only the true positions give a
  smooth field); s scales the field so that max over nodes and components of
  |u| equals the requested amplitude.
* Vectors: x ~ N(0, 1) per DoF.

Layout of every nodal vector: DoF = c * L^d + i + L (j + L k).
"""
import numpy as np

MU_MATRIX = 1.0
NU = 0.3


def lame_lambda(mu, nu=NU):
    return 2.0 * mu * nu / (1.0 - 2.0 * nu)


def two_phase_material(stiff=100.0):
    mu = np.array([MU_MATRIX, stiff * MU_MATRIX])
    lam = np.array([lame_lambda(MU_MATRIX), stiff * lame_lambda(MU_MATRIX)])
    return mu, lam


def two_phase_mu2(stiff=100.0, frac=0.3):
    """Second-invariant moduli of a Mooney-Rivlin variant: frac * mu per phase."""
    return frac * two_phase_material(stiff)[0]


def two_phase_mooney_rivlin(stiff=100.0, frac=0.3):
    """(mu, lambda, mu2) of the Mooney-Rivlin law with the same small-strain
    Lame pair as two_phase_material: mu + mu2 and 2 lambda + 2 mu2 match the
    Neo-Hookean mu and 2 lambda (mu2 = frac * mu)."""
    mu, lam = two_phase_material(stiff)
    mu2 = frac * mu
    return mu - mu2, lam - mu2, mu2


def spheres(n, seed, dim=3, rmin=0.05, rmax=0.12):
    """List of (centre, radius, material_id=1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(r, 1.0 - r, size=dim)
        out.append((c, float(r), 1))
    return out


def _axis(L, coords):
    if coords is None:
        return np.arange(L, dtype=np.float64) / (L - 1)
    t = np.asarray(coords, dtype=np.float64)
    assert t.shape == (L,)
    return t


def sine_field(dim, L, seed, amp, n_modes=8, kmax=2, coords=None):
    """Nodal values (dim * L^dim,) of a smooth seeded displacement field."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n_modes, dim))
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(0, kmax + 1, size=dim)
        if np.any(k):
            ks.append(k)
    ks = np.array(ks, dtype=np.float64)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    t = _axis(L, coords)
    grids = np.meshgrid(*([t] * dim), indexing="ij")
    X = np.stack([g.transpose(tuple(range(dim))[::-1]).reshape(-1) for g in grids], axis=1)
    arg = np.pi * X @ ks.T + phi[None, :]                  # (n_nodes, n_modes)
    u = np.sin(arg) @ a                                    # (n_nodes, dim)
    u *= amp / np.abs(u).max()
    return np.ascontiguousarray(u.T.reshape(-1))


def normal_vector(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


# Dirichlet face-component bits: bit ((2*axis + side) * dim + comp)
def face_bits(dim, axis, side, comps=None):
    comps = range(dim) if comps is None else comps
    m = 0
    for c in comps:
        m |= 1 << ((2 * axis + side) * dim + c)
    return m


def clamp_bottom_top(dim):
    """Both faces normal to the last axis fully constrained."""
    ax = dim - 1
    return face_bits(dim, ax, 0) | face_bits(dim, ax, 1)


def problem(dim, n_cells, degree, n_spheres=0, sphere_seed=3, u_seed=4, u_amp=0.1,
            u_kmax=1, x_seed=5, mask=0, disc=False, n_modes=8):
    """A synthetic problem as plain arrays: mesh sizes, materials, u, x, mask."""
    mu, lam = two_phase_material()
    if disc:
        incl = [(np.full(dim, 0.5), 0.25, 1)]
    else:
        incl = spheres(n_spheres, sphere_seed, dim) if n_spheres else []
    L = degree * n_cells + 1
    u = sine_field(dim, L, u_seed, u_amp, n_modes=n_modes, kmax=u_kmax) if u_amp else np.zeros(dim * L ** dim)
    x = normal_vector(dim * L ** dim, x_seed)
    return dict(dim=dim, n_cells=n_cells, degree=degree, mu=mu, lam=lam,
                inclusions=incl, u=u, x=x, mask=mask)


def square_disc_q1_16():
    """2-D plane-strain unit square, 16x16 Q1, centred disc r = 0.25 (100x stiffer),
    u = 8 seeded sine modes of amplitude 0.05 (seed 1), x ~ N(0,1) (seed 2)."""
    return problem(2, 16, 1, disc=True, u_seed=1, u_amp=0.05, u_kmax=2, x_seed=2)


def cube_spheres_q2(n_cells=32):
    """3-D unit cube, 32^3 Q2, 20 spheres (seed 3, r in [0.05, 0.12]),
    smooth u of amplitude 0.1 (seed 4), x ~ N(0,1) (seed 5)."""
    return problem(3, n_cells, 2, n_spheres=20, sphere_seed=3, u_seed=4, u_amp=0.1,
                   u_kmax=1, x_seed=5)


BATCH_LEVELS = {8: 3, 12: 3, 16: 4, 24: 4}


def batch_of_cubes(n=256, seed=6, sizes=(8, 12, 16, 24), degrees=(1, 2, 3)):
    """256 independent 3-D problems: N uniform in {8, 12, 16, 24} cells per
    direction, degree uniform in {1, 2, 3}, 1-10 spheres (r in [0.05, 0.12]),
    bottom and top clamped.  The linearisation point is a loaded state: a
    uniaxial stretch u_z = e Z with e ~ U[0.02, 0.08] plus a smooth seeded
    perturbation of amplitude e / 20, so max |u| <= 0.1.  Compression turns
    the stress S = mu I - c1 C^-1 indefinite (where J < 1 and a principal
    stretch is short), and with it the tangent, which no CG solve survives:
    random smooth fields of a few percent already do that, and so does a
    perturbation of e / 4 on top of the stretch.  At e / 20 the stress is
    positive definite at every node of all 256 problems.  Returns light
    descriptors; ``batch_fields`` draws the vectors."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = int(rng.choice(sizes))
        p = int(rng.choice(degrees))
        ns = int(rng.integers(1, 11))
        stretch = float(rng.uniform(0.02, 0.08))
        seeds = [int(v) for v in rng.integers(0, 2 ** 31, size=3)]
        out.append(dict(dim=3, n_cells=N, degree=p, n_levels=BATCH_LEVELS.get(N, 1), n_spheres=ns,
                        stretch=stretch, amp=0.05 * stretch, sphere_seed=seeds[0], u_seed=seeds[1],
                        x_seed=seeds[2], mask=clamp_bottom_top(3)))
    return out


def stretched_field(dim, L, stretch, seed, amp, coords=None):
    """u = stretch * X_last e_last + a smooth seeded perturbation (``sine_field``)."""
    u = sine_field(dim, L, seed, amp, kmax=1, coords=coords)
    t = _axis(L, coords)
    u[(dim - 1) * L ** dim:] += stretch * np.repeat(t, L ** (dim - 1))
    return u


def batch_literal_field(desc, coords=None):
    """The batch problem's displacement read literally as a random smooth
    deformation: ``sine_field`` (kmax 1) of amplitude 1.25 * stretch, i.e.
    max |u| in [0.025, 0.1] over the batch.  Such states can make the tangent
    indefinite (no CG solve), which a vmult does not mind."""
    L = desc["degree"] * desc["n_cells"] + 1
    return sine_field(3, L, desc["u_seed"] + 1, 1.25 * desc["stretch"], kmax=1, coords=coords)


def batch_fields(desc, coords=None):
    """(inclusions, u, x) of one problem of the batch; ``coords`` are the support
    points along an axis of its finest level."""
    L = desc["degree"] * desc["n_cells"] + 1
    incl = spheres(desc["n_spheres"], desc["sphere_seed"], 3)
    u = stretched_field(3, L, desc["stretch"], desc["u_seed"], desc["amp"], coords=coords)
    x = normal_vector(3 * L ** 3, desc["x_seed"])
    return incl, u, x
