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

    The prescribed increment dg of a load step enters the first Newton step of
    that step linearly (the paper's Newton system with inhomogeneous
    constraints): K_c d = -(R(u) + K(u) dg) on free rows, u <- u + dg + d.
    Later Newton steps solve K_c du = -R(u).  R0, the reference for the
    relative residual test, is the norm of that first right-hand side.
    Dead tractions (``face_traction``, Sec. 3's Neumann term) scale with the
    load like the prescribed values: R(u) = F_int(u) - s f_ext on free rows.
    The paper does not say what happens when an increment fails; here an
    update that inverts a quadrature point (non-finite residual), a CG
    breakdown (p^T K p <= 0: the tangent is indefinite at the iterate), a CG
    that misses rtol in max_cg steps, or an increment that does not converge
    within max_newton steps is undone and
    the failed increment halved; after a converged cut increment the step
    doubles again up to 1/n_steps.
    """
    mesh = hier.meshes[-1]
    cons = hier.cons[-1]
    free = ~cons
    u = np.zeros(mesh.n_dofs) if u0 is None else np.array(u0, dtype=np.float64)
    f_ext = fe.external_force(mesh, face_traction) if face_traction is not None else np.zeros(mesh.n_dofs)
    f_ext[cons] = 0.0
    records = []
    h0 = 1.0 / n_steps
    done, h, cut = 0.0, h0, 0
    with np.errstate(invalid="ignore"):
        while done < 1.0 - 1e-12:
            target = min(1.0, done + h)
            saved = u.copy()
            g = dirichlet_vector(mesh, face_values, hier.mask, target)
            dg = np.where(cons, g - u, 0.0)
            R0 = None
            conv = False
            for it in range(max_newton):
                R = fe.residual(mesh, hier.mat, u) - target * f_ext
                hier.set_deformation(u)
                b = -R
                if it == 0:
                    b = b - fe.tangent_matrix(mesh, hier.mat, u) @ dg
                b[cons] = 0.0
                nb = np.linalg.norm(b)
                if R0 is None:
                    R0 = nb
                d, cg_it, rel = gmg.pcg(lambda v: hier.A[-1] @ v, b, hier.vcycle, rtol, max_cg)
                if not np.isfinite(rel):          # CG breakdown
                    rec = dict(load_fraction=target, newton=it, res=nb, res_after=np.nan, du=np.nan,
                               cg_iters=cg_it, cg_rel=rel, cutbacks=cut)
                    records.append(rec)
                    if log:
                        log(rec)
                    break
                du = d + dg if it == 0 else d
                u += du
                ndu = np.linalg.norm(du)
                Rn = np.linalg.norm((fe.residual(mesh, hier.mat, u) - target * f_ext)[free])
                rec = dict(load_fraction=target, newton=it, res=nb, res_after=Rn, du=ndu, cg_iters=cg_it,
                           cg_rel=rel, cutbacks=cut)
                records.append(rec)
                if log:
                    log(rec)
                if not np.isfinite(Rn) or rel > rtol:     # inverted, or the linear solve failed
                    break
                if ndu <= du_tol and (Rn <= r_tol or Rn <= r_tol * R0):
                    conv = True
                    break
            if conv:
                done = target
                if h < h0:
                    h = min(h0, 2.0 * h)
                continue
            u = saved
            cut += 1
            if cut > max_cutbacks:
                raise RuntimeError(f"Newton failed after {max_cutbacks} cut-backs at load fraction {done}")
            h = 0.5 * (target - done)
    return u, records
