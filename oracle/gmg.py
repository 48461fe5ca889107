"""Geometric multigrid preconditioned CG (oracle, test infrastructure only).

Sec. 6 builds the level operators by restricting the current displacement to
every multigrid level and linearising there (not by Galerkin products), with
standard geometric transfers between nested Q_p spaces.  Sec. 7 fixes the
remaining settings: a V-cycle with two pre- and two post-smoothing steps of a
degree-4 Chebyshev smoother on the operator diagonal, the smoother interval
[0.6, 1.2] times the largest eigenvalue estimated from 30 CG iterations, and
deal.II's preconditioned CG as the outer solver.

Readings taken where the paper is silent:

* "restrict the displacement" = nodal interpolation of the finer field at the
  coarser support points, applied recursively fine -> coarse (``"nodal"``);
  the alternative ``"vertex"`` takes the values at the coarse cell vertices
  and fills each coarse cell multilinearly;
* the coarse level is solved exactly (dense LU) in FP64, or (``coarse_solver=
  "chebyshev"``, Sec. 7) by the Chebyshev iteration as a solver: interval
  [lambda_min, 1.2 lambda_max] from the coarse level's CG-Lanczos run, degree
  from the bound 1 / T_k <= 1e-3.  Linearised about the
  interpolated displacement, the coarse tangent can be indefinite when the
  coarse mesh does not resolve the material (the assumption of Sec. 6); the
  exact solve is still defined, and ``coarse_negative`` records its number of
  negative eigenvalues;
* the eigenvalue estimate runs Jacobi-preconditioned CG on A y = r0 with r0
  drawn from SplitMix64 (``oracle.rng``, seed ``EIG_SEED``) in [-1, 1) and
  zeroed on constrained DoFs; the largest eigenvalue of the Lanczos
  tridiagonal built from the CG coefficients is the estimate;
* Dirichlet DoFs carry identity rows: transfers zero them, the diagonal is 1.

Everything here is FP64 and uses assembled scipy matrices; it is built for
clarity, not speed.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import basis, fe, rng

EIG_SEED = 0x5EED


# --- transfers -------------------------------------------------------------------

def _eval_global_1d(mesh_from, X):
    """M[k, I] = global 1-D basis function of lattice node I of ``mesh_from``
    evaluated at coordinate X[k]."""
    p, N, h = mesh_from.p, mesh_from.N, mesh_from.h
    M = np.zeros((len(X), mesh_from.L))
    for k, x in enumerate(X):
        e = min(int(np.floor(x / h)), N - 1)
        t = (x - e * h) / h
        V, _ = basis.lagrange(mesh_from.xi, [t])
        M[k, p * e: p * e + p + 1] = V[0]
    M[np.abs(M) < 1e-15] = 0.0
    return M


def prolongation_1d(coarse, fine):
    """P1[I_f, I_c] = phi^coarse_{I_c}(X_f)."""
    return _eval_global_1d(coarse, fine.coords_1d())


def interpolation_1d(fine, coarse):
    """I1[I_c, I_f] = phi^fine_{I_f}(X_c)."""
    return _eval_global_1d(fine, coarse.coords_1d())


def vertex_interpolation_1d(fine, coarse):
    """V1[I_c, I_f]: the coarse node's value is the linear interpolant, along
    the axis, of the fine field's values at the two vertices of the coarse cell
    that holds it (the vertices are fine lattice nodes)."""
    Xf, Xc = fine.coords_1d(), coarse.coords_1d()
    hc = 1.0 / coarse.N
    V = np.zeros((len(Xc), len(Xf)))
    for k, x in enumerate(Xc):
        e = min(int(np.floor(x / hc + 1e-12)), coarse.N - 1)
        t = (x - e * hc) / hc
        lo = int(np.argmin(np.abs(Xf - e * hc)))
        hi = int(np.argmin(np.abs(Xf - (e + 1) * hc)))
        V[k, lo] += 1.0 - t
        V[k, hi] += t
    V[np.abs(V) < 1e-15] = 0.0
    return V


def _tensor(M1, d):
    """Tensor-product operator on node vectors (node = i + L j + L^2 k), applied
    per component (block diagonal over the d components)."""
    M1 = sp.csr_matrix(M1)
    T = M1
    for _ in range(d - 1):
        T = sp.kron(M1, T)           # slower axis on the left
    return sp.block_diag([T] * d).tocsr()


def prolongation(coarse, fine):
    return _tensor(prolongation_1d(coarse, fine), fine.d)


def interpolation(fine, coarse, level_field="nodal"):
    M1 = interpolation_1d(fine, coarse) if level_field == "nodal" else vertex_interpolation_1d(fine, coarse)
    return _tensor(M1, fine.d)


# --- smoother pieces -------------------------------------------------------------

def diagonal(A_c):
    """Diagonal of the constrained operator (1 on constrained DoFs)."""
    return A_c.diagonal().copy()


def chebyshev(apply_A, dinv, f, x, lo, hi, degree):
    """Degree-``degree`` Chebyshev iteration for D^-1 A on [lo, hi]
    (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 12.1,
    with the residual preconditioned by D^-1 and recomputed each step)."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = np.array(x, dtype=np.float64, copy=True)
    r = f - apply_A(x)
    d = dinv * r / theta
    x += d
    for _ in range(degree - 1):
        r = f - apply_A(x)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * dinv * r
        x += d
        rho = rho_new
    return x


class BreakdownError(RuntimeError):
    """CG met p^T A p <= 0 (the operator is not positive definite) before the
    eigenvalue estimate had a single step."""


def lanczos_lambda_max(apply_A, dinv, r0, iters):
    """Largest eigenvalue of D^-1 A estimated from ``iters`` steps of
    Jacobi-preconditioned CG on A y = r0, through the CG-Lanczos relation
    (Saad, Sec. 6.7.3): T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    T_{j,j+1} = sqrt(beta_j)/alpha_j."""
    r = np.array(r0, dtype=np.float64, copy=True)
    z = dinv * r
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for _ in range(iters):
        Ap = apply_A(p)
        pAp = p @ Ap
        if not pAp > 0.0:
            break
        alpha = rz / pAp
        r = r - alpha * Ap
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        alphas.append(alpha)
        betas.append(beta)
        if rz_new <= 0.0:
            break
        p = z + beta * p
        rz = rz_new
    m = len(alphas)
    if m == 0:
        raise BreakdownError("eigenvalue estimate: the first CG step met p^T A p <= 0")
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    ev = np.linalg.eigvalsh(T)
    lanczos_lambda_max.last_min = float(ev.min())    # smallest Ritz value of the same run
    return float(ev.max()), m


COARSE_REDUCTION = 1e-3     # Sec. 7: the coarse Chebyshev solver reduces the residual by 10^3


def chebyshev_solver_degree(lo, hi, eps):
    """Smallest k with 1 / T_k((hi + lo) / (hi - lo)) <= eps (the Chebyshev
    iteration's error bound on [lo, hi]), at most 1000."""
    if not (lo > 0 and hi > lo):
        raise ValueError("the Chebyshev coarse solver needs 0 < lambda_min < lambda_max")
    k = np.arccosh(1.0 / eps) / np.arccosh((hi + lo) / (hi - lo))
    return int(min(1000, max(1, np.ceil(k))))


def eig_start_vector(n, constrained):
    r0 = rng.uniform_pm1(EIG_SEED, n)
    r0[constrained] = 0.0
    return r0


# --- hierarchy -------------------------------------------------------------------

class Hierarchy:
    """Levels 0 (coarsest) .. n_levels-1 (finest) of a uniformly refined box.

    ``n_coarse`` cells per direction on level 0; level l has n_coarse * 2^l.
    """

    def __init__(self, dim, n_coarse, degree, n_levels, mat, mask=0,
                 cheb_degree=4, n_smooth=2, eig_iters=30, cheb_lo=0.6, cheb_hi=1.2, level_field="nodal",
                 coarse_solver="direct"):
        self.meshes = [fe.Mesh(dim, n_coarse * 2 ** l, degree) for l in range(n_levels)]
        self.mat = mat
        self.mask = mask
        self.cons = [m.constrained(mask) for m in self.meshes]
        self.P = [None] + [prolongation(self.meshes[l - 1], self.meshes[l]) for l in range(1, n_levels)]
        self.I = [None] + [interpolation(self.meshes[l], self.meshes[l - 1], level_field) for l in range(1, n_levels)]
        self.cheb_degree = cheb_degree
        self.n_smooth = n_smooth
        self.eig_iters = eig_iters
        self.cheb_lo, self.cheb_hi = cheb_lo, cheb_hi
        self.coarse_solver = coarse_solver

    @property
    def n_levels(self):
        return len(self.meshes)

    def level_displacements(self, u_fine):
        us = [None] * self.n_levels
        us[-1] = np.asarray(u_fine, dtype=np.float64)
        for l in range(self.n_levels - 1, 0, -1):
            us[l - 1] = self.I[l] @ us[l]
        return us

    def set_deformation(self, u_fine):
        self.us = self.level_displacements(u_fine)
        self.A, self.dinv, self.lam_max, self.interval = [], [], [], []
        for l, m in enumerate(self.meshes):
            K = fe.tangent_matrix(m, self.mat, self.us[l])
            A = fe.constrain_matrix(K, self.cons[l])
            self.A.append(A)
            dinv = 1.0 / diagonal(A)
            self.dinv.append(dinv)
            if l > 0 or self.coarse_solver == "chebyshev":
                lmax, _ = lanczos_lambda_max(lambda v, A=A: A @ v, dinv,
                                             eig_start_vector(m.n_dofs, self.cons[l]),
                                             self.eig_iters)
                lmin = lanczos_lambda_max.last_min
            else:
                lmax = lmin = np.nan
            self.lam_max.append(lmax)
            if l == 0 and self.coarse_solver == "chebyshev":
                self.lam_min0 = lmin
                self.interval.append((lmin, self.cheb_hi * lmax))
                self.coarse_degree = chebyshev_solver_degree(lmin, self.cheb_hi * lmax, COARSE_REDUCTION)
            else:
                self.interval.append((self.cheb_lo * lmax, self.cheb_hi * lmax))
        A0 = self.A[0].toarray()
        self.coarse = sla.lu_factor(A0)
        self._A0 = A0

    @property
    def coarse_negative(self):
        """Number of negative eigenvalues of the coarse tangent (dense eigensolver)."""
        return int((np.linalg.eigvalsh(self._A0) < 0).sum())

    def smooth(self, l, f, x):
        lo, hi = self.interval[l]
        A = self.A[l]
        for _ in range(self.n_smooth):
            x = chebyshev(lambda v: A @ v, self.dinv[l], f, x, lo, hi, self.cheb_degree)
        return x

    def vcycle(self, r, l=None):
        """One V-cycle applied to the residual r on level l (default finest)."""
        l = self.n_levels - 1 if l is None else l
        if l == 0:
            if self.coarse_solver == "chebyshev":
                lo, hi = self.interval[0]
                return chebyshev(lambda v: self.A[0] @ v, self.dinv[0], r, np.zeros_like(r), lo, hi,
                                 self.coarse_degree)
            return sla.lu_solve(self.coarse, r)
        x = self.smooth(l, r, np.zeros_like(r))
        rc = self.P[l].T @ (r - self.A[l] @ x)
        rc[self.cons[l - 1]] = 0.0
        e = self.P[l] @ self.vcycle(rc, l - 1)
        e[self.cons[l]] = 0.0
        x = x + e
        return self.smooth(l, r, x)


def pcg(apply_A, b, precond, rtol, max_it):
    """Preconditioned CG (Hestenes-Stiefel), x0 = 0, stop at |r|/|b| <= rtol.

    Returns (x, iterations, relative residual); the relative residual is NaN
    when CG breaks down (p^T A p <= 0, which an SPD operator never gives).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    z = precond(r)
    p = z.copy()
    rz = r @ z
    it = 0
    rel = 1.0
    while it < max_it:
        Ap = apply_A(p)
        pAp = p @ Ap
        it += 1
        if not pAp > 0.0:
            return x, it, np.nan
        alpha = rz / pAp
        x += alpha * p
        r -= alpha * Ap
        rel = np.linalg.norm(r) / nb
        if rel <= rtol:
            break
        z = precond(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, rel
