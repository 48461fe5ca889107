"""Compressible Neo-Hookean material law (oracle, test infrastructure only).

Sec. 2.3 defines the strain energy per unit reference volume

    psi(C) = mu/2 [tr C - tr I - 2 ln J] + lambda ln^2 J,   J = sqrt(det C),

and prints its first and second derivatives with respect to C.  The energy is
implemented exactly as printed (note: lambda ln^2 J, without a factor 1/2, so
the small-strain limit is linear elasticity with Lame pair (mu, 2 lambda)).

The oracle's operator route is *referential*:

    S   = 2 dpsi/dC        = mu I - c1 C^-1,              c1 = mu - 2 lambda ln J
    CC  = 4 d2psi/dCdC     = 2 c1 I_{C^-1} + 2 lambda C^-1 (x) C^-1
          with (I_{C^-1})_{IJKL} = 1/2 (Ci_IK Ci_JL + Ci_IL Ci_JK)
    P   = F S                                    (first Piola-Kirchhoff)
    A   = dP/dF,  A_{iIkL} = delta_ik S_IL + F_iJ F_kK CC_{JIKL}

The spatial closed forms of Sec. 2.3 (tau = mu b - c1 I and
J*c = 2 c1 Ssym + 2 lambda I (x) I, with its cheap action) are provided
separately (``tau_closed_form``, ``jc_closed_form``) so that tests can check
the push-forward identities tau = chi(S) and J*c = chi(CC) (Sec. 2.1) instead
of assuming them.  All arrays may carry leading batch dimensions; the last
two (or four) axes are tensor indices.
"""
import numpy as np


def psi(F, mu, lam):
    """Strain energy psi(C(F)) of Sec. 2.3; F has shape (..., d, d)."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    C = np.einsum("...kI,...kJ->...IJ", F, F)
    J = np.linalg.det(F)
    lnJ = np.log(J)
    trC = np.trace(C, axis1=-2, axis2=-1)
    return 0.5 * mu * (trC - d - 2.0 * lnJ) + lam * lnJ ** 2


def pk2(F, mu, lam):
    """Second Piola-Kirchhoff stress S = 2 dpsi/dC = mu I - c1 C^-1."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    C = np.einsum("...kI,...kJ->...IJ", F, F)
    Ci = np.linalg.inv(C)
    J = np.linalg.det(F)
    c1 = mu - 2.0 * lam * np.log(J)
    mu_b = np.asarray(mu, dtype=np.float64)
    return mu_b[..., None, None] * np.eye(d) - c1[..., None, None] * Ci


def referential_tangent(F, mu, lam):
    """CC = 4 d2psi/dC dC = 2 c1 I_{C^-1} + 2 lambda C^-1 (x) C^-1 (Sec. 2.3).

    The first term is 4 * 1/2 c1 (-dC^-1/dC) with the minor-symmetric form
    (-dC^-1/dC)_{IJKL} = 1/2 (Ci_IK Ci_JL + Ci_IL Ci_JK).
    """
    F = np.asarray(F, dtype=np.float64)
    C = np.einsum("...kI,...kJ->...IJ", F, F)
    Ci = np.linalg.inv(C)
    J = np.linalg.det(F)
    c1 = mu - 2.0 * lam * np.log(J)
    sym = 0.5 * (np.einsum("...IK,...JL->...IJKL", Ci, Ci)
                 + np.einsum("...IL,...JK->...IJKL", Ci, Ci))
    outer = np.einsum("...IJ,...KL->...IJKL", Ci, Ci)
    lam_b = np.asarray(lam, dtype=np.float64)
    return 2.0 * c1[..., None, None, None, None] * sym \
        + 2.0 * lam_b[..., None, None, None, None] * outer


def pk1(F, mu, lam):
    """First Piola-Kirchhoff stress P = F S."""
    return np.einsum("...iJ,...JI->...iI", F, pk2(F, mu, lam))


def dP_dF(F, mu, lam):
    """A_{iIkL} = dP_iI / dF_kL = delta_ik S_IL + F_iJ F_kK CC_{JIKL}."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    S = pk2(F, mu, lam)
    CC = referential_tangent(F, mu, lam)
    geo = np.einsum("ik,...IL->...iIkL", np.eye(d), S)
    mat = np.einsum("...iJ,...kK,...JIKL->...iIkL", F, F, CC, optimize=True)
    return geo + mat


# --- spatial closed forms printed in Sec. 2.3 (used only as independent pins) ---

def tau_closed_form(F, mu, lam):
    """Kirchhoff stress as printed: tau = mu b - [mu - 2 lambda ln J] I."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    b = np.einsum("...iK,...jK->...ij", F, F)
    c1 = mu - 2.0 * lam * np.log(np.linalg.det(F))
    mu_b = np.asarray(mu, dtype=np.float64)
    return mu_b[..., None, None] * b - c1[..., None, None] * np.eye(d)


def jc_closed_form(F, mu, lam):
    """Material part of the spatial tangent as printed:
    J*c = 2 [mu - 2 lambda ln J] Ssym + 2 lambda I (x) I,
    with Ssym_{ijkl} = 1/2 (delta_ik delta_jl + delta_il delta_jk)."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    eye = np.eye(d)
    c1 = mu - 2.0 * lam * np.log(np.linalg.det(F))
    ssym = 0.5 * (np.einsum("ik,jl->ijkl", eye, eye) + np.einsum("il,jk->ijkl", eye, eye))
    ii = np.einsum("ij,kl->ijkl", eye, eye)
    lam_b = np.asarray(lam, dtype=np.float64)
    return 2.0 * c1[..., None, None, None, None] * ssym + 2.0 * lam_b[..., None, None, None, None] * ii


def jc_action(F, mu, lam, G):
    """Cheap action of J*c on a symmetric tensor G, as printed in Sec. 2.3:
    J*c : G = 2 [mu - 2 lambda ln J] G + 2 lambda tr(G) I."""
    d = F.shape[-1]
    c1 = mu - 2.0 * lam * np.log(np.linalg.det(F))
    tr = np.trace(G, axis1=-2, axis2=-1)
    return 2.0 * c1[..., None, None] * G + 2.0 * np.asarray(lam)[..., None, None] * tr[..., None, None] * np.eye(d)


def push_forward2(F, A):
    """chi(A)_ij = F_iA A_AB F_jB (Sec. 2.1)."""
    return np.einsum("...iA,...AB,...jB->...ij", F, A, F)


def push_forward4(F, A):
    """chi(A)_ijkl = F_iA F_jB A_ABCD F_kC F_lD (Sec. 2.1)."""
    return np.einsum("...iA,...jB,...ABCD,...kC,...lD->...ijkl", F, F, A, F, F)
