"""Pins of the closed-form solvation energies: the value printed in the
paper, the Born ion, the Kelvin image limit and explicit Bessel functions."""
import json
import math
import os

import numpy as np
import pytest

from oracle import analytic as A

GOLD = os.path.join(os.path.dirname(__file__), "golden", "kirkwood_sphere.json")


def test_kirkwood_matches_printed_value():
    g = json.load(open(GOLD))
    e = A.kirkwood_energy(g["radius"], g["charge_xyz"], [g["charge_q"]], g["eps1"], g["eps2"], g["kappa"])
    assert e == pytest.approx(g["energy_kcal_per_mol"], rel=5e-7)


def test_kirkwood_centre_is_born():
    for kap in (0.0, 0.125, 1.0):
        e = A.kirkwood_energy(3.0, [0, 0, 0], [1.5], 2.0, 80.0, kap)
        b = A.born_energy(3.0, 1.5, 2.0, 80.0, kap)
        assert e == pytest.approx(b, rel=1e-13)
    # Born closed form itself, written from the charging-work picture:
    # dG = q^2/2 * (1/(eps2 a (1+ka)) - 1/(eps1 a)) * 332.0637
    assert A.born_energy(4, 1, 4, 80, 0.125) == pytest.approx(-10.0310909375, rel=1e-12)


def test_no_dielectric_jump_no_energy():
    e = A.kirkwood_energy(4.0, [[1, 1, 1], [-1, 0.5, 0]], [1.0, -0.7], 4.0, 4.0, 0.0)
    assert abs(e) < 1e-12


@pytest.mark.parametrize("kappa", [0.0, 0.3])
def test_conductor_limit_is_kelvin_image(kappa):
    """eps2 -> infinity: grounded sphere; the reaction potential is that of
    the Kelvin image charge -q a/s at distance a^2/s from the centre."""
    a, s, q, eps1 = 4.0, 1.7, 1.3, 2.0
    e = A.kirkwood_energy(a, [0, 0, s], [q], eps1, 1e13, kappa, nmax=120)
    image = -0.5 * q * q * a / (eps1 * (a * a - s * s)) * A.KCAL_PER_MOL
    assert e == pytest.approx(image, rel=1e-9)


def test_bessel_ratio_against_explicit_functions():
    """k0 = e^-x/x, k1 = e^-x (1/x + 1/x^2), k2 = e^-x (1/x + 3/x^2 + 3/x^3)."""
    x = 0.73
    fns = [lambda t: math.exp(-t) / t,
           lambda t: math.exp(-t) * (1 / t + 1 / t ** 2),
           lambda t: math.exp(-t) * (1 / t + 3 / t ** 2 + 3 / t ** 3)]
    R = A._bessel_k_ratio(2, x)
    h = 1e-6
    for n, f in enumerate(fns):
        d = (f(x + h) - f(x - h)) / (2 * h)
        assert R[n] == pytest.approx(x * d / f(x), rel=1e-8)
