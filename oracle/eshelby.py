"""Eshelby's interior solution for an ellipsoidal inclusion in an infinite
isotropic body (the verification problem of Sec. 4.1: an ellipsoid with
semi-axes a = (a1, a2, a3) carrying a uniform eigenstrain eps* inside, the
same moduli inside and out).  TEST INFRASTRUCTURE ONLY: used by tests/ to
check the solver's interior displacement, never by the product path.

Inside the ellipsoid the strain is uniform, eps = S : eps*, with S the
Eshelby tensor; for an ellipsoid centred at the origin and aligned with the
axes the displacement is u_i = eps_ij x_j there.  S is written in terms of
the potential integrals of the ellipsoid (Eshelby 1957; the I-integral form
of Mura's *Micromechanics of defects in solids*, Sec. 11):

    I_i  = 2 pi a1 a2 a3 Int_0^inf ds / ((a_i^2 + s) D(s))
    I_ij = 2 pi a1 a2 a3 Int_0^inf ds / ((a_i^2 + s)(a_j^2 + s) D(s))
    D(s) = sqrt((a1^2 + s)(a2^2 + s)(a3^2 + s))

which this module evaluates by adaptive quadrature of the definitions, and

    S_iiii = 3 a_i^2 I_ii / (8 pi (1-nu)) + (1-2nu) I_i / (8 pi (1-nu))
    S_iijj = a_j^2 I_ij / (8 pi (1-nu)) - (1-2nu) I_i / (8 pi (1-nu))      (i != j)
    S_ijij = S_ijji = (a_i^2 + a_j^2) I_ij / (16 pi (1-nu))
                      + (1-2nu) (I_i + I_j) / (16 pi (1-nu))                 (i != j)

(no summation), every other component zero.  The paper compares against the
explicit field of a later reference that is not reproduced here; the
interior solution above is the classical one that field reduces to inside
the inclusion.  Pins (tests/test_oracle_pins.py): the sphere's textbook
values, the elliptic cylinder's (a3 -> infinity), the prolate spheroid's
elementary closed form of I_i, and the shape-independent dilatation
S_iikk = (1+nu)/(1-nu).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate


def potential_integrals(a):
    """(I, II): I[i] = I_i and II[i, j] = I_ij of the ellipsoid with
    semi-axes a, each by quadrature of its defining integral, taken over
    log(s) (s = e^tau, ds = s dtau) from s = 1e-14 min(a)^2 to 1e14 max(a)^2
    with break points at log(a_i^2): the integrand is smooth in tau and the
    two cut-off tails are below 1e-13 of the integral."""
    a = np.asarray(a, dtype=np.float64)
    assert a.shape == (3,) and np.all(a > 0)
    a2 = a * a
    pref = 2.0 * np.pi * a[0] * a[1] * a[2]
    lo = np.log(1e-14 * a2.min())
    hi = np.log(1e14 * a2.max())
    brk = sorted(set(np.log(a2)))

    def quad(weight):
        def f(tau):
            s = np.exp(tau)
            D = np.sqrt((a2[0] + s) * (a2[1] + s) * (a2[2] + s))
            return weight(s) / D * s
        v, err = integrate.quad(f, lo, hi, points=brk, epsabs=0.0, epsrel=1e-13, limit=1000)
        return pref * v

    I = np.array([quad(lambda s, i=i: 1.0 / (a2[i] + s)) for i in range(3)])
    II = np.empty((3, 3))
    for i in range(3):
        for j in range(i, 3):
            II[i, j] = II[j, i] = quad(lambda s, i=i, j=j: 1.0 / ((a2[i] + s) * (a2[j] + s)))
    return I, II


def eshelby_tensor(a, nu):
    """Eshelby tensor S[i, j, k, l] (3x3x3x3) of the ellipsoid a in an
    isotropic body with Poisson ratio nu, from the I-integrals above."""
    a = np.asarray(a, dtype=np.float64)
    I, II = potential_integrals(a)
    a2 = a * a
    c = 1.0 / (8.0 * np.pi * (1.0 - nu))
    S = np.zeros((3, 3, 3, 3))
    for i in range(3):
        S[i, i, i, i] = 3.0 * c * a2[i] * II[i, i] + c * (1.0 - 2.0 * nu) * I[i]
        for j in range(3):
            if j == i:
                continue
            S[i, i, j, j] = c * a2[j] * II[i, j] - c * (1.0 - 2.0 * nu) * I[i]
            v = 0.5 * c * (a2[i] + a2[j]) * II[i, j] + 0.5 * c * (1.0 - 2.0 * nu) * (I[i] + I[j])
            S[i, j, i, j] = S[i, j, j, i] = v
    return S


def interior_strain(a, nu, eps_star):
    """Uniform strain inside the inclusion: eps_ij = S_ijkl eps*_kl."""
    S = eshelby_tensor(a, nu)
    return np.einsum("ijkl,kl->ij", S, np.asarray(eps_star, dtype=np.float64))


def interior_displacement(a, nu, eps_star, x, y, z):
    """u_i = eps_ij x_j inside the inclusion (centred at the origin, axes
    along x, y, z; the rigid motion is zero by symmetry).  Shape (3, ...)."""
    e = interior_strain(a, nu, eps_star)
    X = np.broadcast_arrays(x, y, z)
    return np.stack([e[i, 0] * X[0] + e[i, 1] * X[1] + e[i, 2] * X[2] for i in range(3)])
