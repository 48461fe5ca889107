"""Finite-element discretisation of the Neo-Hookean body (oracle, test
infrastructure only).

Discretisation (Sec. 3 and Sec. 5):

* The body is the unit box [0,1]^d (d = 2: plane strain, d = 3), split into
  N^d equal cells of size h = 1/N.
* The displacement is a vector-valued continuous Lagrange field of degree p on
  each cell, with Gauss-Lobatto-Legendre support points; the global nodes form
  a lattice of L = pN+1 points per direction.
* Numbering (tensor multi-index of Sec. 5 / Fig. 2, first index fastest):
  node = i + L (j + L k); DoF = c * L^d + node for component c.  Inside a cell,
  local node a = a_x + n (a_y + n a_z) with n = p+1, and quadrature point
  q = q_x + n_q (q_y + n_q q_z); cells are numbered e = e_x + N (e_y + N e_z).
* Integration uses the tensor-product Gauss rule with q = p+1 points per
  direction (Tables 1 and 2) in the referential configuration.

The discrete residual and tangent are those of eq. (linear_system) /
eq. (algebraic_tangent), evaluated here in the referential route:

    R_(a,i)         = sum_K sum_q w_q h^d  P_iI  dN_a/dX_I
    K_(a,i),(b,k)   = sum_K sum_q w_q h^d  dN_a/dX_I A_iIkL dN_b/dX_L

with P = F S and A = dP/dF from ``oracle.material``.  The matrix-free vmult of
eq. (mf_vmult) reaches exactly this matrix when it uses the same quadrature,
so the oracle vmult is the assembled matrix times the vector.

Dirichlet conditions fix whole components on whole faces; the constrained
operator is K_c = (I - C) K (I - C) + C with C the indicator of constrained
DoFs, and the constrained residual has zero constrained rows.
"""
import numpy as np
import scipy.sparse as sp

from . import basis, material


class Mesh:
    """Structured Q_p lattice on the unit box with N cells per direction."""

    def __init__(self, dim, n_cells, degree):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        self.d = int(dim)
        self.N = int(n_cells)
        self.p = int(degree)
        self.n = self.p + 1                   # support points per direction
        self.nq1 = self.p + 1                 # Gauss points per direction
        self.L = self.p * self.N + 1
        self.h = 1.0 / self.N
        self.n_nodes = self.L ** self.d
        self.n_dofs = self.d * self.n_nodes
        self.n_cells = self.N ** self.d
        self.nA = self.n ** self.d            # nodes per cell
        self.nQ = self.nq1 ** self.d          # quadrature points per cell
        self.xi = basis.gll_points(self.p)
        self.gx, self.gw = basis.gauss_rule(self.nq1)
        self.S1, self.D1 = basis.lagrange(self.xi, self.gx)   # (nq1, n)
        self._build_reference_tables()

    # -- reference-cell tables ------------------------------------------------
    def _multi(self, idx, base):
        out = []
        for _ in range(self.d):
            out.append(idx % base)
            idx //= base
        return out

    def _build_reference_tables(self):
        d, n, nq = self.d, self.n, self.nq1
        G = np.zeros((self.nQ, self.nA, d))
        Wq = np.zeros(self.nQ)
        for q in range(self.nQ):
            qm = self._multi(q, nq)
            Wq[q] = np.prod([self.gw[qm[k]] for k in range(d)])
            for a in range(self.nA):
                am = self._multi(a, n)
                for I in range(d):
                    val = 1.0
                    for k in range(d):
                        tab = self.D1 if k == I else self.S1
                        val *= tab[qm[k], am[k]]
                    G[q, a, I] = val / self.h
        self.G = G                            # dN_a/dX_I at qp q (physical)
        self.W = Wq * self.h ** d             # w_q * |cell|
        qpos = np.zeros((self.nQ, d))
        for q in range(self.nQ):
            qm = self._multi(q, nq)
            qpos[q] = [self.gx[qm[k]] for k in range(d)]
        self.qref = qpos                      # qp position inside a cell, in [0,1]^d
        apos = np.zeros((self.nA, d), dtype=np.int64)
        for a in range(self.nA):
            apos[a] = self._multi(a, n)
        self.aoff = apos                      # local node lattice offsets

    # -- lattice ---------------------------------------------------------------
    def coords_1d(self):
        """Reference coordinate of every lattice index along one axis."""
        I = np.arange(self.L)
        e = np.minimum(I // self.p, self.N - 1)
        a = I - self.p * e
        return self.h * (e + self.xi[a])

    def node_coords(self):
        """(n_nodes, d) reference coordinates of all nodes, node order."""
        x1 = self.coords_1d()
        grids = np.meshgrid(*([x1] * self.d), indexing="ij")
        # node = i + L j + L^2 k  -> axis 0 of the flattened index is the slowest
        cols = [g.transpose(tuple(range(self.d))[::-1]).reshape(-1) for g in grids]
        return np.stack(cols, axis=1)

    def all_cells(self):
        return np.arange(self.n_cells)

    def cell_index(self, cells):
        cells = np.asarray(cells, dtype=np.int64)
        return np.stack(self._multi(cells.copy(), self.N), axis=1)   # (nc, d)

    def cell_nodes(self, cells):
        cm = self.cell_index(cells)                                    # (nc, d)
        lat = self.p * cm[:, None, :] + self.aoff[None, :, :]          # (nc, nA, d)
        node = np.zeros(lat.shape[:2], dtype=np.int64)
        for k in reversed(range(self.d)):
            node = node * self.L + lat[:, :, k]
        return node

    def cell_dofs(self, cells):
        nodes = self.cell_nodes(cells)
        comps = np.arange(self.d, dtype=np.int64)[None, :, None] * self.n_nodes
        return comps + nodes[:, None, :]                               # (nc, d, nA)

    def qp_coords(self, cells):
        cm = self.cell_index(cells).astype(np.float64)
        return self.h * (cm[:, None, :] + self.qref[None, :, :])       # (nc, nQ, d)

    def cells_of_node(self, node):
        """Cells whose closure contains the lattice node."""
        lat = []
        nd = int(node)
        for _ in range(self.d):
            lat.append(nd % self.L)
            nd //= self.L
        per_axis = []
        for I in lat:
            cand = {I // self.p, (I - 1) // self.p} if I % self.p == 0 else {I // self.p}
            per_axis.append(sorted(c for c in cand if 0 <= c < self.N))
        out = []
        for combo in np.array(np.meshgrid(*per_axis, indexing="ij")).reshape(self.d, -1).T:
            e = 0
            for k in reversed(range(self.d)):
                e = e * self.N + int(combo[k])
            out.append(e)
        return out

    def constrained(self, mask):
        """Boolean DoF indicator for a face-component mask.

        Bit ((2*axis + side) * d + comp) set means component ``comp`` is fixed
        on the face ``axis`` = 0 (side 0) or ``axis`` = 1 (side 1).
        """
        c = np.zeros(self.n_dofs, dtype=bool)
        if not mask:
            return c
        lat = np.indices((self.L,) * self.d).reshape(self.d, -1)[::-1]   # lat[axis][node]
        for axis in range(self.d):
            for side in range(2):
                on_face = lat[axis] == (0 if side == 0 else self.L - 1)
                for comp in range(self.d):
                    if (mask >> ((2 * axis + side) * self.d + comp)) & 1:
                        c[comp * self.n_nodes + np.nonzero(on_face)[0]] = True
        return c


class Material:
    """Piecewise-constant material parameters.

    ``mu[m]``, ``lam[m]`` for material m (0 = matrix); ``mu2[m]`` the
    second-invariant modulus of the Mooney-Rivlin law (zero: Neo-Hookean).  ``inclusions`` is a list
    of (centre, radius, material_id); a point X belongs to an inclusion when
    |X - centre|^2 <= radius^2, later inclusions overriding earlier ones.  The
    indicator is sampled at every quadrature point's reference position on
    every level (the paper resolves inclusions with the coarse mesh; synthetic
    spheres are not mesh-aligned).
    """

    def __init__(self, mu, lam, inclusions=(), mu2=None):
        self.mu = np.asarray(mu, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.mu2 = np.zeros_like(self.mu) if mu2 is None else np.asarray(mu2, dtype=np.float64)
        self.inclusions = [(np.asarray(c, dtype=np.float64), float(r), int(m))
                           for (c, r, m) in inclusions]

    def ids_at(self, X):
        X = np.asarray(X, dtype=np.float64)
        ids = np.zeros(X.shape[:-1], dtype=np.int64)
        for c, r, m in self.inclusions:
            inside = np.sum((X - c[: X.shape[-1]]) ** 2, axis=-1) <= r * r
            ids[inside] = m
        return ids

    def params(self, mesh, cells):
        ids = self.ids_at(mesh.qp_coords(cells))
        return self.mu[ids], self.lam[ids]                             # (nc, nQ)

    def mu2_at(self, mesh, cells):
        return self.mu2[self.ids_at(mesh.qp_coords(cells))]


# --- element kernels -----------------------------------------------------------

def deformation_gradient(mesh, u, cells):
    """F = I + Grad u at every quadrature point of ``cells`` -> (nc, nQ, d, d)."""
    ue = np.asarray(u, dtype=np.float64)[mesh.cell_dofs(cells)]       # (nc, d, nA)
    H = np.einsum("cia,qaI->cqiI", ue, mesh.G)
    return H + np.eye(mesh.d)


def element_residual(mesh, mat, u, cells):
    F = deformation_gradient(mesh, u, cells)
    mu, lam = mat.params(mesh, cells)
    P = material.pk1(F, mu, lam, mat.mu2_at(mesh, cells))
    return np.einsum("q,qaI,cqiI->cia", mesh.W, mesh.G, P)            # (nc, d, nA)


def element_tangent(mesh, mat, u, cells):
    """K_e[c, i, a, k, b] = sum_q w_q G[q, a, I] A[c, q, i, I, k, L] G[q, b, L].

    Evaluated as two contractions (trial gradient first, then one matrix
    product over the pair (q, I)); the single four-operand einsum computes the
    same sum in another order and is two orders of magnitude slower at degree 4.
    """
    F = deformation_gradient(mesh, u, cells)
    mu, lam = mat.params(mesh, cells)
    A = material.dP_dF(F, mu, lam, mat.mu2_at(mesh, cells))           # (nc, nQ, d, d, d, d)
    nc, nq, d = A.shape[0], A.shape[1], A.shape[2]
    nA = mesh.G.shape[1]
    AG = np.einsum("cqiIkL,qbL->cqiIkb", A, mesh.G)                    # (nc, nQ, d, d, d, nA)
    X = AG.transpose(0, 2, 1, 3, 4, 5).reshape(nc, d, nq * d, d * nA)  # sum index (q, I)
    WG = (mesh.W[:, None, None] * mesh.G).transpose(1, 0, 2).reshape(nA, nq * d)
    return np.matmul(WG, X).reshape(nc, d, nA, d, nA)


def _cell_chunk(mesh, chunk):
    """Cells per chunk, bounded so that one chunk's intermediates stay near 256 MB."""
    per_cell = mesh.G.shape[0] * mesh.d ** 3 * mesh.G.shape[1] * 8
    return max(1, min(chunk, (1 << 28) // per_cell))


def _chunks(n, size):
    for s in range(0, n, size):
        yield np.arange(s, min(n, s + size))


def residual(mesh, mat, u, constrained=None, chunk=2048):
    """Global residual R (eq. linear_system, volume part); constrained rows zeroed."""
    R = np.zeros(mesh.n_dofs)
    for cells in _chunks(mesh.n_cells, chunk):
        Re = element_residual(mesh, mat, u, cells)
        np.add.at(R, mesh.cell_dofs(cells).reshape(-1), Re.reshape(-1))
    if constrained is not None:
        R[constrained] = 0.0
    return R


def external_force(mesh, face_traction):
    """Nodal external force f_a = sum over loaded faces of the integral of
    T_f N_a over the face (the Neumann term of the weak form, Sec. 3), for
    dead (reference-configuration) tractions: face_traction[2*axis + side][comp].

    Each face is integrated cell face by cell face with the face's own Gauss
    rule (q = p + 1 points per direction) on the restricted shape functions.
    """
    d, p, L = mesh.d, mesh.p, mesh.L
    f = np.zeros(mesh.n_dofs)
    lat = np.indices((L,) * d).reshape(d, -1)[::-1]               # lattice index per node, axis-major
    gx, gw = basis.gauss_rule(p + 1)
    V, _ = basis.lagrange(mesh.xi, gx)                            # (q, p + 1) values on [0, 1]
    # 1-D face-cell integrals of each local basis function: int_0^h phi_b = h sum_q w_q V[q, b]
    m1 = mesh.h * (gw @ V)                                        # (p + 1,)
    for axis in range(d):
        for side in range(2):
            t = np.asarray(face_traction[2 * axis + side], dtype=np.float64)
            if not np.any(t):
                continue
            on_face = np.nonzero(lat[axis] == (0 if side == 0 else L - 1))[0]
            tang = [a for a in range(d) if a != axis]
            for node in on_face:
                # the node's weight: sum over the face cells containing it of the
                # product of the 1-D integrals of its basis function per tangential axis
                w = 1.0
                for a in tang:
                    I = lat[a][node]
                    wa = 0.0
                    for e in range(mesh.N):
                        b = I - p * e
                        if 0 <= b <= p:
                            wa += m1[b]
                    w *= wa
                for c in range(d):
                    f[c * mesh.n_nodes + node] += t[c] * w
    return f


def tangent_matrix(mesh, mat, u, chunk=1024):
    """Assembled (unconstrained) tangent as scipy CSR."""
    nd = mesh.d * mesh.nA
    rows, cols, vals = [], [], []
    for cells in _chunks(mesh.n_cells, _cell_chunk(mesh, chunk)):
        Ke = element_tangent(mesh, mat, u, cells).reshape(len(cells), nd, nd)
        dofs = mesh.cell_dofs(cells).reshape(len(cells), nd)
        rows.append(np.repeat(dofs, nd, axis=1).reshape(-1))
        cols.append(np.tile(dofs, (1, nd)).reshape(-1))
        vals.append(Ke.reshape(-1))
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(mesh.n_dofs, mesh.n_dofs))
    return K.tocsr()


def constrain_matrix(K, constrained):
    """K_c = (I - C) K (I - C) + C."""
    free = sp.diags((~constrained).astype(np.float64))
    return (free @ K @ free + sp.diags(constrained.astype(np.float64))).tocsr()


def vmult_ebe(mesh, mat, u, x, constrained=None, cells=None, chunk=512):
    """Element-by-element y = K_c x (same element matrices as the assembly)."""
    x = np.asarray(x, dtype=np.float64)
    xm = x.copy()
    if constrained is not None:
        xm[constrained] = 0.0
    y = np.zeros(mesh.n_dofs)
    cells_all = mesh.all_cells() if cells is None else np.asarray(cells)
    nd = mesh.d * mesh.nA
    chunk = _cell_chunk(mesh, chunk)
    for s in range(0, len(cells_all), chunk):
        cells = cells_all[s:s + chunk]
        Ke = element_tangent(mesh, mat, u, cells).reshape(len(cells), nd, nd)
        dofs = mesh.cell_dofs(cells).reshape(len(cells), nd)
        ye = np.einsum("cij,cj->ci", Ke, xm[dofs])
        np.add.at(y, dofs.reshape(-1), ye.reshape(-1))
    if constrained is not None:
        y[constrained] = x[constrained]
    return y


def vmult_rows(mesh, mat, u, x, rows, constrained=None):
    """Selected entries (K_c x)[rows], each from the cells around its node."""
    x = np.asarray(x, dtype=np.float64)
    xm = x.copy()
    if constrained is not None:
        xm[constrained] = 0.0
    out = np.zeros(len(rows))
    nd = mesh.d * mesh.nA
    for r_i, r in enumerate(rows):
        if constrained is not None and constrained[r]:
            out[r_i] = x[r]
            continue
        node = r % mesh.n_nodes
        cells = np.array(mesh.cells_of_node(node))
        Ke = element_tangent(mesh, mat, u, cells).reshape(len(cells), nd, nd)
        dofs = mesh.cell_dofs(cells).reshape(len(cells), nd)
        ye = np.einsum("cij,cj->ci", Ke, xm[dofs])
        out[r_i] = ye[dofs == r].sum()
    return out


def residual_rows(mesh, mat, u, rows, constrained=None):
    """Selected entries of the constrained residual."""
    out = np.zeros(len(rows))
    for r_i, r in enumerate(rows):
        if constrained is not None and constrained[r]:
            continue
        node = r % mesh.n_nodes
        cells = np.array(mesh.cells_of_node(node))
        Re = element_residual(mesh, mat, u, cells)
        out[r_i] = Re[mesh.cell_dofs(cells) == r].sum()
    return out


def min_jacobian(mesh, u, chunk=4096):
    """Smallest det F over all quadrature points."""
    mj = np.inf
    for cells in _chunks(mesh.n_cells, chunk):
        mj = min(mj, float(np.linalg.det(deformation_gradient(mesh, u, cells)).min()))
    return mj
