"""TEDOPA chain mapping: the chain coefficients of a bosonic bath (host).

Sec. III, Eqs. (def-sd), (chainmap), (H_1D): a bath of spectral density
J(omega) on [0, omega_c] (dispersion g(x) = x) becomes a chain whose
frequencies and hoppings are the recurrence coefficients of the orthogonal
polynomials of the measure J(omega)/pi d omega.  Here the measure is
discretised by an M-point Gauss-Legendre rule and its Jacobi matrix (the
tridiagonal matrix of the recurrence) is built by the Lanczos process on
diag(nodes) started from the square roots of the weights, with full
reorthogonalisation (one of the stable procedures the paper refers to):
  omega_n = a_n (diagonal), t_n = b_{n+1} (off-diagonal, between chain
  oscillators n and n+1), t_0 = sqrt(mass) (coupling of the system).
Model preparation only: the result feeds models.spin_boson_chain.
"""
import numpy as np


def ohmic(alpha, s, omega_c):
    """J(omega) = 2 pi alpha omega_c (omega / omega_c)^s on [0, omega_c]."""
    return lambda w: 2.0 * np.pi * alpha * omega_c * (np.asarray(w) / omega_c) ** s


def chain_coefficients(J, omega_c, n_modes, points=4000):
    """(t0, omegas[n_modes], hoppings[n_modes - 1]) of the mapped chain."""
    x, w = np.polynomial.legendre.leggauss(int(points))
    nodes = 0.5 * omega_c * (x + 1.0)
    weights = 0.5 * omega_c * w * J(nodes) / np.pi
    mass = float(np.sum(weights))
    m = int(n_modes)
    Q = np.zeros((m, len(nodes)))
    q = np.sqrt(weights / mass)
    diag = np.zeros(m)
    off = np.zeros(max(m - 1, 0))
    for k in range(m):
        Q[k] = q
        v = nodes * q
        diag[k] = q @ v
        if k + 1 == m:
            break
        v = v - diag[k] * q - (off[k - 1] * Q[k - 1] if k > 0 else 0.0)
        for _ in range(2):                       # full reorthogonalisation, twice
            v = v - Q[:k + 1].T @ (Q[:k + 1] @ v)
        off[k] = np.linalg.norm(v)
        q = v / off[k]
    return float(np.sqrt(mass)), diag, off
