"""Compressible Neo-Hookean material law and a Mooney-Rivlin variant (oracle,
test infrastructure only).

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

A second law, compressible Mooney-Rivlin, shows that the tensor4 route of
Sec. 5 (Algorithm 3: cache the material part of the spatial tangent and the
stress) does not depend on the constitutive law.  It adds a second-invariant
term with modulus mu2 and keeps the paper's conventions (stress-free
reference, lambda ln^2 J):

    psi = mu/2 [I1 - 3 - 2 ln J] + mu2/2 [I2 - 3 - 4 ln J] + lambda ln^2 J,
    S   = mu (I - C^-1) + mu2 (I1 I - C - 2 C^-1) + 2 lambda ln J C^-1,
    CC  = 2 c1' I_{C^-1} + 2 lambda C^-1 (x) C^-1 + 2 mu2 (I (x) I - Ssym),
          c1' = mu + 2 mu2 - 2 lambda ln J,

with I1, I2 the invariants of the 3-D C (plane strain: C_33 = 1, so
I1 = tr C + 1 and I2 = (I1^2 - tr C^2 - 1) / 2 for the 2x2 block).  mu2 = 0 is
the Neo-Hookean law above; the small-strain limit has Lame pair
(mu + mu2, 2 lambda + 2 mu2).  Every function below takes mu2 (default 0).

The spatial closed forms of Sec. 2.3 (tau = mu b - c1 I and
J*c = 2 c1 Ssym + 2 lambda I (x) I, with its cheap action) are provided
separately (``tau_closed_form``, ``jc_closed_form``) so that tests can check
the push-forward identities tau = chi(S) and J*c = chi(CC) (Sec. 2.1) instead
of assuming them.  All arrays may carry leading batch dimensions; the last
two (or four) axes are tensor indices.
"""
import numpy as np


def _has_mu2(mu2):
    return np.any(np.asarray(mu2) != 0.0)


def invariants(C):
    """I1, I2 of the 3-D right Cauchy-Green tensor whose leading d x d block
    is C (plane strain for d = 2: C_33 = 1)."""
    d = C.shape[-1]
    I1 = np.trace(C, axis1=-2, axis2=-1) + (3 - d)
    trC2 = np.einsum("...IJ,...JI->...", C, C) + (3 - d)
    return I1, 0.5 * (I1 ** 2 - trC2)


def psi(F, mu, lam, mu2=0.0):
    """Strain energy psi(C(F)) of Sec. 2.3 (plus the Mooney-Rivlin term);
    F has shape (..., d, d)."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    C = np.einsum("...kI,...kJ->...IJ", F, F)
    J = np.linalg.det(F)
    lnJ = np.log(J)
    trC = np.trace(C, axis1=-2, axis2=-1)
    out = 0.5 * mu * (trC - d - 2.0 * lnJ) + lam * lnJ ** 2
    if _has_mu2(mu2):
        _, I2 = invariants(C)
        out = out + 0.5 * mu2 * (I2 - 3.0 - 4.0 * lnJ)
    return out


def pk2(F, mu, lam, mu2=0.0):
    """Second Piola-Kirchhoff stress S = 2 dpsi/dC = mu I - c1 C^-1
    (+ mu2 (I1 I - C - 2 C^-1))."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    C = np.einsum("...kI,...kJ->...IJ", F, F)
    Ci = np.linalg.inv(C)
    J = np.linalg.det(F)
    c1 = mu - 2.0 * lam * np.log(J)
    mu_b = np.asarray(mu, dtype=np.float64)
    S = mu_b[..., None, None] * np.eye(d) - c1[..., None, None] * Ci
    if _has_mu2(mu2):
        I1, _ = invariants(C)
        m2 = np.asarray(mu2, dtype=np.float64)[..., None, None]
        S = S + m2 * (I1[..., None, None] * np.eye(d) - C - 2.0 * Ci)
    return S


def referential_tangent(F, mu, lam, mu2=0.0):
    """CC = 4 d2psi/dC dC = 2 c1 I_{C^-1} + 2 lambda C^-1 (x) C^-1 (Sec. 2.3)
    (+ 2 mu2 (2 I_{C^-1} + I (x) I - Ssym)).

    The first term is 4 * 1/2 c1 (-dC^-1/dC) with the minor-symmetric form
    (-dC^-1/dC)_{IJKL} = 1/2 (Ci_IK Ci_JL + Ci_IL Ci_JK).
    """
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    C = np.einsum("...kI,...kJ->...IJ", F, F)
    Ci = np.linalg.inv(C)
    J = np.linalg.det(F)
    c1 = mu - 2.0 * lam * np.log(J)
    sym = 0.5 * (np.einsum("...IK,...JL->...IJKL", Ci, Ci)
                 + np.einsum("...IL,...JK->...IJKL", Ci, Ci))
    outer = np.einsum("...IJ,...KL->...IJKL", Ci, Ci)
    lam_b = np.asarray(lam, dtype=np.float64)
    CC = 2.0 * c1[..., None, None, None, None] * sym \
        + 2.0 * lam_b[..., None, None, None, None] * outer
    if _has_mu2(mu2):
        eye = np.eye(d)
        ssym = 0.5 * (np.einsum("IK,JL->IJKL", eye, eye) + np.einsum("IL,JK->IJKL", eye, eye))
        ii = np.einsum("IJ,KL->IJKL", eye, eye)
        m2 = np.asarray(mu2, dtype=np.float64)[..., None, None, None, None]
        CC = CC + 2.0 * m2 * (2.0 * sym + ii - ssym)
    return CC


def pk1(F, mu, lam, mu2=0.0):
    """First Piola-Kirchhoff stress P = F S."""
    return np.einsum("...iJ,...JI->...iI", F, pk2(F, mu, lam, mu2))


def dP_dF(F, mu, lam, mu2=0.0):
    """A_{iIkL} = dP_iI / dF_kL = delta_ik S_IL + F_iJ F_kK CC_{JIKL}."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    S = pk2(F, mu, lam, mu2)
    CC = referential_tangent(F, mu, lam, mu2)
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


# --- spatial closed forms of the Mooney-Rivlin law (derived; pins for the push-forwards) ---

def mr_tau_closed_form(F, mu, lam, mu2):
    """tau = F S F^T = mu (b - I) + mu2 (I1 b - b^2 - 2 I) + 2 lambda ln J I."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    b = np.einsum("...iK,...jK->...ij", F, F)
    I1, _ = invariants(b)
    lnJ = np.log(np.linalg.det(F))
    eye = np.eye(d)
    return mu * (b - eye) + mu2 * (I1[..., None, None] * b - b @ b - 2.0 * eye) \
        + 2.0 * lam * lnJ[..., None, None] * eye


def mr_jc_closed_form(F, mu, lam, mu2):
    """J*c = 2 c1' Ssym + 2 lambda I (x) I + 2 mu2 (b (x) b - I_b),
    c1' = mu + 2 mu2 - 2 lambda ln J, (I_b)_{ijkl} = 1/2 (b_ik b_jl + b_il b_jk)."""
    F = np.asarray(F, dtype=np.float64)
    d = F.shape[-1]
    b = np.einsum("...iK,...jK->...ij", F, F)
    eye = np.eye(d)
    c1p = mu + 2.0 * mu2 - 2.0 * lam * np.log(np.linalg.det(F))
    ssym = 0.5 * (np.einsum("ik,jl->ijkl", eye, eye) + np.einsum("il,jk->ijkl", eye, eye))
    ii = np.einsum("ij,kl->ijkl", eye, eye)
    bb = np.einsum("ij,kl->ijkl", b, b)
    ib = 0.5 * (np.einsum("ik,jl->ijkl", b, b) + np.einsum("il,jk->ijkl", b, b))
    return 2.0 * c1p * ssym + 2.0 * lam * ii + 2.0 * mu2 * (bb - ib)


def push_forward2(F, A):
    """chi(A)_ij = F_iA A_AB F_jB (Sec. 2.1)."""
    return np.einsum("...iA,...AB,...jB->...ij", F, A, F)


def push_forward4(F, A):
    """chi(A)_ijkl = F_iA F_jB A_ABCD F_kC F_lD (Sec. 2.1)."""
    return np.einsum("...iA,...jB,...ABCD,...kC,...lD->...ijkl", F, F, A, F, F)
