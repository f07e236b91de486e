"""Closed-form solvation energies used as pins (Results: mesh refinement
study with an analytical solution; Methods: reaction potential and polar
solvation energy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Units: lengths in Angstrom, charges in e, energies in kcal/mol.  The
electrostatic conversion constant 332.0637 kcal A / (mol e^2) is a reading:
the paper does not print it.

Kirkwood's sphere (dielectric sphere of radius a, permittivity eps1 inside,
eps2 and inverse Debye length kappa outside, point charges inside): expand
the Coulomb potential of each charge in Legendre modes about the centre,
write the interior reaction potential as a regular solid harmonic series and
the exterior potential with modified spherical Bessel functions k_n(kappa r),
and impose continuity of phi and eps dphi/dr at r = a for every mode.  With
x = kappa a and R_n = x k_n'(x) / k_n(x) the reaction coefficient of mode n
for a charge q at distance s from the centre is
   B_n a^n = q s^n / a^(n+1) * [(n+1) + (eps2/eps1) R_n] / (eps1 n - eps2 R_n)
and phi_reac(r) = sum_n B_n a^n (|r|/a)^n P_n(cos gamma) (gamma the angle
between r and the charge).  The polar solvation energy is
   dG = 1/2 sum_k q_k phi_reac(r_k).
For n = 0 this is the Born ion, (q^2 / 2a) [1/(eps2 (1 + kappa a)) - 1/eps1].
"""
from __future__ import annotations

import numpy as np

KCAL_PER_MOL = 332.0637  # e^2/A -> kcal/mol (reading, not printed in the paper)


def born_energy(a: float, q: float, eps1: float, eps2: float, kappa: float) -> float:
    """Born ion with salt: charge q at the centre of a sphere of radius a."""
    return 0.5 * KCAL_PER_MOL * q * q / a * (1.0 / (eps2 * (1.0 + kappa * a)) - 1.0 / eps1)


def _bessel_k_ratio(nmax: int, x: float) -> np.ndarray:
    """R_n = x k_n'(x)/k_n(x) for n = 0..nmax (modified spherical Bessel
    functions of the second kind).  Uses rho_n = k_{n-1}/k_n with rho_0 = 1,
    rho_{n+1} = 1 / (rho_n + (2n+1)/x) (from k_{n+1} = k_{n-1} + (2n+1)/x k_n)
    and k_n' = -k_{n-1} - (n+1)/x k_n.  For x = 0, R_n = -(n+1)."""
    n = np.arange(nmax + 1, dtype=np.float64)
    if x == 0.0:
        return -(n + 1.0)
    rho = np.empty(nmax + 1)
    rho[0] = 1.0
    for k in range(nmax):
        rho[k + 1] = 1.0 / (rho[k] + (2 * k + 1) / x)
    return -x * rho - (n + 1.0)


def _legendre(nmax: int, c):
    c = np.asarray(c, dtype=np.float64)
    P = np.empty((nmax + 1,) + c.shape)
    P[0] = 1.0
    if nmax >= 1:
        P[1] = c
    for n in range(1, nmax):
        P[n + 1] = ((2 * n + 1) * c * P[n] - n * P[n - 1]) / (n + 1)
    return P


def kirkwood_reaction_potential(a, charges_xyz, charges_q, eval_xyz, eps1, eps2, kappa,
                                nmax: int = 60):
    """phi_reac (e/A units, i.e. before the kcal/mol factor) at eval points
    inside the sphere centred at the origin."""
    xq = np.atleast_2d(np.asarray(charges_xyz, dtype=np.float64))
    qq = np.atleast_1d(np.asarray(charges_q, dtype=np.float64))
    xe = np.atleast_2d(np.asarray(eval_xyz, dtype=np.float64))
    R = _bessel_k_ratio(nmax, kappa * a)
    n = np.arange(nmax + 1, dtype=np.float64)
    coef = ((n + 1) + (eps2 / eps1) * R) / (eps1 * n - eps2 * R)
    out = np.zeros(len(xe))
    for k in range(len(xq)):
        s = np.linalg.norm(xq[k])
        for i in range(len(xe)):
            re = np.linalg.norm(xe[i])
            if s == 0.0 or re == 0.0:
                cosg = 1.0
            else:
                cosg = float(np.dot(xq[k], xe[i]) / (s * re))
            P = _legendre(nmax, cosg)
            out[i] += np.sum(qq[k] * s ** n / a ** (n + 1) * coef * (re / a) ** n * P)
    return out


def kirkwood_energy(a, charges_xyz, charges_q, eps1, eps2, kappa, nmax: int = 60) -> float:
    """Polar solvation energy (kcal/mol) of point charges inside a sphere of
    radius a centred at the origin."""
    xq = np.atleast_2d(np.asarray(charges_xyz, dtype=np.float64))
    qq = np.atleast_1d(np.asarray(charges_q, dtype=np.float64))
    phi = kirkwood_reaction_potential(a, xq, qq, xq, eps1, eps2, kappa, nmax)
    return 0.5 * KCAL_PER_MOL * float(np.dot(qq, phi))
