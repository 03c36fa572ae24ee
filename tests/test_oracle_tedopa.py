"""Pins of the TEDOPA chain-mapping oracle (oracle/tedopa.py).

For J(omega) = 2 pi alpha omega_c (omega/omega_c)^s on [0, omega_c] the
measure J/pi is, up to its mass, the Jacobi weight x^s on [0, 1] scaled by
omega_c, whose monic recurrence is a textbook closed form (Jacobi
polynomials P^(0,s) moved from [-1, 1] to [0, 1]):
  a_n = omega_c (1 + s^2 / ((2n + s)(2n + s + 2))) / 2,
  b_n = omega_c^2 n^2 (n + s)^2 / ((2n + s)^2 (2n + s + 1)(2n + s - 1)), n >= 1,
  b_0 = mass = 2 alpha omega_c^2 / (s + 1).
The discretised Stieltjes procedure must reproduce it; a wrong recurrence
index, a dropped term or a wrong normalisation fails here.
"""
import numpy as np
import pytest

from oracle import tedopa


def _jacobi(n, s, omega_c, alpha):
    k = np.arange(n, dtype=np.float64)
    a = 0.5 * omega_c * (1.0 + s * s / ((2 * k + s) * (2 * k + s + 2)))
    b = np.zeros(n)
    kk = k[1:]
    b[1:] = omega_c ** 2 * kk ** 2 * (kk + s) ** 2 / ((2 * kk + s) ** 2 * (2 * kk + s + 1) * (2 * kk + s - 1))
    b[0] = 2.0 * alpha * omega_c ** 2 / (s + 1.0)
    return a, b


@pytest.mark.parametrize("s,omega_c,alpha", [(1.0, 1.0, 0.1), (0.5, 3.0, 0.2), (2.0, 1.0, 0.05)])
def test_stieltjes_matches_jacobi_recurrence(s, omega_c, alpha):
    n = 80
    J = tedopa.ohmic(alpha, s, omega_c)
    x, w = tedopa.discretised_measure(J, omega_c, 6000)
    a, b = tedopa.stieltjes(x, w, n)
    ea, eb = _jacobi(n, s, omega_c, alpha)
    tol = 1e-11 if s == int(s) else 5e-6    # omega^0.5 is not polynomial: quadrature error
    assert np.max(np.abs(a - ea)) < tol * omega_c
    assert np.max(np.abs(b[1:] - eb[1:])) < tol * omega_c ** 2
    assert abs(b[0] - eb[0]) < tol * eb[0]


def test_chain_coefficients_and_their_limits():
    # hoppings tend to omega_c / 4 and frequencies to omega_c / 2 (the
    # asymptotics of any measure on [0, omega_c] with Jacobi-type ends)
    t0, om, t = tedopa.chain_coefficients(tedopa.ohmic(0.1, 1.0, 2.0), 2.0, 120)
    assert abs(t0 - np.sqrt(2 * 0.1 * 4.0 / 2.0)) < 1e-12
    assert len(om) == 120 and len(t) == 119
    assert abs(om[-1] - 1.0) < 1e-4 and abs(t[-1] - 0.5) < 1e-4


def test_general_chain_reduces_to_uniform_chain():
    # with constant coefficients the TEDOPA Hamiltonian is the uniform chain
    from oracle import models
    dims = [2, 4, 4, 4]
    a = models.spin_boson_chain(4, 4, 1.0, 0.5, 1.0, 0.5)[1]
    b = models.spin_boson_chain_general(dims, 1.0, 0.5, [1.0] * 3, [0.5] * 2)[1]
    for x, y in zip(a, b):
        assert np.max(np.abs(x - y)) < 1e-15
