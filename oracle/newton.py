"""Newton-Raphson load stepping with the GMG-preconditioned CG (oracle, test
infrastructure only).

Sec. 3 solves A du = -F for the Newton correction; Sec. 7 applies the load in
steps and stops Newton when the l2 norm of the update is below 1e-5 and the
residual is below 1e-8 in absolute or relative terms.  The load here is
displacement control: constant prescribed values per constrained face
component, scaled linearly over the load steps.
"""
import numpy as np

from . import fe, gmg

# Step length (the paper does not globalise its Newton method): an update is
# scaled by 1, 1/2, 1/4, ... (at most MAX_HALVINGS halvings) until the trial
# state keeps J > 0 at every quadrature point (a finite residual) and, once
# the prescribed values are met, the squared residual norm drops by the
# Armijo factor 1 - 2 ARMIJO alpha (the merit function |R|^2 / 2 falls at
# rate |R|^2 along an exact Newton direction).
MAX_HALVINGS = 12
ARMIJO = 1e-4


def dirichlet_vector(mesh, face_values, mask, scale=1.0):
    """Vector holding the prescribed values on constrained DoFs (zero elsewhere).

    ``face_values[2*axis + side][comp]`` is the value on that face; where two
    constrained faces meet the face listed later in axis-major order wins.
    """
    g = np.zeros(mesh.n_dofs)
    lat = np.indices((mesh.L,) * mesh.d).reshape(mesh.d, -1)[::-1]
    for axis in range(mesh.d):
        for side in range(2):
            on_face = np.nonzero(lat[axis] == (0 if side == 0 else mesh.L - 1))[0]
            for comp in range(mesh.d):
                if (mask >> ((2 * axis + side) * mesh.d + comp)) & 1:
                    g[comp * mesh.n_nodes + on_face] = scale * face_values[2 * axis + side][comp]
    return g


def solve(hier, face_values, n_steps, rtol=1e-8, max_cg=200, du_tol=1e-5,
          r_tol=1e-8, max_newton=20, u0=None, log=None, max_cutbacks=8, face_traction=None):
    """Full Newton solve; returns (u, records) with one record per Newton step.

    While the prescribed values g of the current load fraction are not yet met
    (the first Newton step of an increment, and after a shortened step that
    carried only part of them), a Newton step carries the remainder
    dg = g - u on constrained DoFs linearly (the paper's Newton system with
    inhomogeneous constraints): K_c d = -(R(u) + K(u) dg) on free rows, update
    du = dg + d.  Otherwise it solves K_c d = -R(u), du = d.  R0, the
    reference for the relative residual test, is the norm of the increment's
    first right-hand side.  The update is u <- u + alpha du with the step
    length alpha of MAX_HALVINGS / ARMIJO above; a full step sets the
    constrained entries to g exactly.
    Dead tractions (``face_traction``, Sec. 3's Neumann term) scale with the
    load like the prescribed values: R(u) = F_int(u) - s f_ext on free rows.
    The paper does not say what happens when an increment fails; here an
    increment fails on a CG breakdown (p^T K p <= 0: the tangent is indefinite
    at the iterate, also when it stops the smoother's eigenvalue estimate at
    its first step), a CG that misses rtol in max_cg steps, an update for
    which no step length is accepted, or when max_newton steps do not
    converge.  The failed increment is undone and halved, down to
    1/2^max_cutbacks of a load step (the solve fails when an increment of that
    size fails); after a converged cut increment the step doubles again up to
    1/n_steps.
    """
    mesh = hier.meshes[-1]
    cons = hier.cons[-1]
    free = ~cons
    u = np.zeros(mesh.n_dofs) if u0 is None else np.array(u0, dtype=np.float64)
    f_ext = fe.external_force(mesh, face_traction) if face_traction is not None else np.zeros(mesh.n_dofs)
    f_ext[cons] = 0.0
    records = []
    h0 = 1.0 / n_steps
    done, h, total_cut = 0.0, h0, 0

    def res(v, s):
        return fe.residual(mesh, hier.mat, v) - s * f_ext

    with np.errstate(invalid="ignore", divide="ignore"):
        while done < 1.0 - 1e-12:
            target = min(1.0, done + h)
            saved = u.copy()
            g = dirichlet_vector(mesh, face_values, hier.mask, target)
            R0 = None
            conv = False
            pending = True                     # prescribed values not yet met
            R = res(u, target)
            for it in range(max_newton):
                try:
                    hier.set_deformation(u)
                except gmg.BreakdownError:        # a level tangent too indefinite to estimate
                    records.append(dict(load_fraction=target, newton=it, res=np.nan, res_after=np.nan,
                                        du=np.nan, cg_iters=0, cg_rel=np.nan, cutbacks=total_cut, alpha=np.nan))
                    if log:
                        log(records[-1])
                    break
                b = -R
                dg = np.where(cons, g - u, 0.0) if pending else np.zeros(mesh.n_dofs)
                if pending:
                    b = b - fe.tangent_matrix(mesh, hier.mat, u) @ dg
                b[cons] = 0.0
                nb = np.linalg.norm(b)
                if R0 is None:
                    R0 = nb
                d, cg_it, rel = gmg.pcg(lambda v: hier.A[-1] @ v, b, hier.vcycle, rtol, max_cg)
                rec = dict(load_fraction=target, newton=it, res=nb, res_after=np.nan, du=np.nan,
                           cg_iters=cg_it, cg_rel=rel, cutbacks=total_cut, alpha=np.nan)
                if not np.isfinite(rel) or rel > rtol:          # CG breakdown or no convergence
                    records.append(rec)
                    if log:
                        log(rec)
                    break
                du = d + dg
                r2 = np.linalg.norm(R[free]) ** 2
                alpha, accepted = 1.0, False
                for _ in range(MAX_HALVINGS + 1):
                    ut = u + alpha * du
                    if alpha == 1.0 and pending:
                        ut[cons] = g[cons]
                    Rt = res(ut, target)
                    rt = np.linalg.norm(Rt[free])
                    if np.isfinite(rt) and (pending or rt * rt <= (1.0 - 2.0 * ARMIJO * alpha) * r2):
                        accepted = True
                        break
                    alpha *= 0.5
                if not accepted:
                    records.append(rec)
                    if log:
                        log(rec)
                    break
                ndu = alpha * np.linalg.norm(du)
                u, R = ut, Rt
                pending = pending and alpha < 1.0
                rec.update(res_after=rt, du=ndu, alpha=alpha)
                records.append(rec)
                if log:
                    log(rec)
                if not pending and ndu <= du_tol and (rt <= r_tol or rt <= r_tol * R0):
                    conv = True
                    break
            if conv:
                done = target
                if h < h0:
                    h = min(h0, 2.0 * h)
                continue
            u = saved
            total_cut += 1
            if target - done <= h0 / 2 ** max_cutbacks * (1.0 + 1e-9):
                raise RuntimeError(f"Newton failed: an increment of 1/{2 ** max_cutbacks} of a load step did not "
                                   f"converge at load fraction {done}")
            h = 0.5 * (target - done)
    return u, records
