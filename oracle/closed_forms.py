"""Closed-form effective stiffnesses used to pin the oracle (small strain).

All matrices use the macro index convention of the solver: Voigt order with
engineering shear strains, C_IJ = E_I : C : E_J with E_I the unit macro tensors
(shear units carry 1/2 in both off-diagonal entries).
"""

import numpy as np


def _units(d):
    pairs = {2: [(0, 0), (1, 1), (0, 1)], 3: [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]}[d]
    out = []
    for i, j in pairs:
        E = np.zeros((d, d))
        if i == j:
            E[i, i] = 1.0
        else:
            E[i, j] = E[j, i] = 0.5
        out.append(E)
    return out


def isotropic_tensor(lam, mu, d):
    """C_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk)."""
    I = np.eye(d)
    return (lam * np.einsum("ij,kl->ijkl", I, I)
            + mu * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)))


def to_matrix(C4):
    d = C4.shape[0]
    U = _units(d)
    return np.array([[np.einsum("ij,ijkl,kl->", EI, C4, EJ) for EJ in U] for EI in U])


def isotropic_matrix(lam, mu, d):
    return to_matrix(isotropic_tensor(lam, mu, d))


def voigt_reuss(C_list, fractions):
    """Voigt (arithmetic) and Reuss (harmonic) averages of stiffness matrices."""
    f = np.asarray(fractions, dtype=np.float64)
    CV = sum(fi * Ci for fi, Ci in zip(f, C_list))
    SR = sum(fi * np.linalg.inv(Ci) for fi, Ci in zip(f, C_list))
    return CV, np.linalg.inv(SR)


def laminate(C4_list, fractions, normal):
    """Exact effective stiffness of a rank-one laminate.

    Per phase p with layer normal n: the strain is E + sym(a_p (x) n), the
    traction (C_p : strain) n is the same vector t in every layer, and the
    jumps a_p average to zero.  With A_p = n.C_p.n and s_p = (C_p:E) n:
    a_p = A_p^-1 (t - s_p),  t = (sum f A^-1)^-1 sum f A^-1 s_p.
    """
    n = np.asarray(normal, dtype=np.float64)
    d = n.shape[0]
    f = np.asarray(fractions, dtype=np.float64)
    A = [np.einsum("j,ijkl,l->ik", n, C, n) for C in C4_list]
    Ainv = [np.linalg.inv(a) for a in A]
    M = np.linalg.inv(sum(fi * ai for fi, ai in zip(f, Ainv)))
    U = _units(d)
    m = len(U)
    out = np.zeros((m, m))
    for J, E in enumerate(U):
        s = [np.einsum("ijkl,kl,j->i", C, E, n) for C in C4_list]
        t = M @ sum(fi * ai @ si for fi, ai, si in zip(f, Ainv, s))
        sigma = np.zeros((d, d))
        for fi, C, ai, si in zip(f, C4_list, Ainv, s):
            a = ai @ (t - si)
            strain = E + 0.5 * (np.outer(a, n) + np.outer(n, a))
            sigma += fi * np.einsum("ijkl,kl->ij", C, strain)
        for I, EI in enumerate(U):
            out[I, J] = np.sum(sigma * EI)
    return out


def eshelby_dilute_disk(lam_m, mu_m, lam_i, mu_i, fraction):
    """Dilute (non-interacting) estimate for circular fibres in plane strain.

    Uses Eshelby's interior tensor of a circular cylinder in an isotropic
    matrix with Poisson ratio nu: on the plane-strain bulk part
    s_J = 1 / (2 (1 - nu)), on the deviatoric part s_K = (3 - 4 nu) / (4 (1 - nu)).
    The strain concentration is A = [I + S C_m^-1 (C_i - C_m)]^-1 and
    C = C_m + f (C_i - C_m) A, exact to first order in the fraction f.
    """
    nu = lam_m / (2.0 * (lam_m + mu_m))
    sJ = 1.0 / (2.0 * (1.0 - nu))
    sK = (3.0 - 4.0 * nu) / (4.0 * (1.0 - nu))
    km, ki = lam_m + mu_m, lam_i + mu_i
    aJ = 1.0 / (1.0 + sJ * (ki - km) / km)
    aK = 1.0 / (1.0 + sK * (mu_i - mu_m) / mu_m)
    k = km + fraction * (ki - km) * aJ
    m = mu_m + fraction * (mu_i - mu_m) * aK
    return np.array([[k + m, k - m, 0.0], [k - m, k + m, 0.0], [0.0, 0.0, m]])
