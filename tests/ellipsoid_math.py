"""Depolarisation factors of an ellipsoid (test helper, no method arithmetic).

The field inside a uniformly charged ellipsoid of semi-axes (a_1, a_2, a_3) and density rho is
linear, E_i = rho n_i x_i / eps0, with
n_i = (a_1 a_2 a_3 / 2) int_0^inf ds / ((s + a_i^2) sqrt((s + a_1^2)(s + a_2^2)(s + a_3^2))),
sum_i n_i = 1 (classical electrostatics of the ellipsoid).
"""
import numpy as np
from scipy import integrate


def depolarisation(semi):
    # n_i depends on the axis ratios only: integrate on the ellipsoid scaled to unit longest axis
    u = np.asarray(semi, dtype=float)
    u = u / u.max()
    a2 = u ** 2
    root = lambda s: np.sqrt(np.prod(s + a2))
    return np.array([0.5 * np.prod(u) * integrate.quad(
        lambda s, i=i: 1.0 / ((s + a2[i]) * root(s)), 0, np.inf, epsabs=0, epsrel=1e-12)[0]
        for i in range(3)])
