"""TEDOPA chain mapping (oracle side): chain coefficients of a bath.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper: Sec. III, Eqs. (def-sd), (chainmap) and (H_1D).  A bath with
spectral density J(omega) on [0, omega_c] (dispersion g(x) = x, so the
measure of Eq. (chainmap) is d mu(omega) = J(omega) / pi d omega) is mapped
by the orthogonal polynomials of that measure to a semi-infinite chain.
With the monic three-term recurrence
    pi_{n+1}(x) = (x - a_n) pi_n(x) - b_n pi_{n-1}(x),  b_0 = mu([0, omega_c]),
the chain of Eq. (H_1D) has on-site frequencies omega_n = a_n, hoppings
t_n = sqrt(b_{n+1}) between oscillators n and n+1, and the system coupling
t_0 = sqrt(b_0) (the paper names Gautschi's numerically stable procedures
for the recurrence; this oracle takes the discretised Stieltjes procedure
on a Gauss-Legendre rule).

Pinned in tests by the closed-form recurrence of the Jacobi polynomials for
J(omega) proportional to omega^s with a hard cut-off.
"""
import numpy as np
import scipy.special


def ohmic(alpha, s, omega_c):
    """J(omega) = 2 pi alpha omega_c (omega / omega_c)^s on [0, omega_c]."""
    return lambda w: 2.0 * np.pi * alpha * omega_c * (np.asarray(w) / omega_c) ** s


def discretised_measure(J, omega_c, points):
    """Gauss-Legendre nodes on [0, omega_c] with weights of J / pi."""
    x, w = scipy.special.roots_legendre(points)
    nodes = 0.5 * omega_c * (x + 1.0)
    weights = 0.5 * omega_c * w * J(nodes) / np.pi
    return nodes, weights


def stieltjes(nodes, weights, n):
    """First n recurrence coefficients (a_k, b_k) of the discrete measure by
    the Stieltjes procedure (inner products of the monic polynomials)."""
    a = np.zeros(n)
    b = np.zeros(n)
    p_prev = np.zeros_like(nodes)
    p = np.ones_like(nodes)
    norm_prev = 1.0
    for k in range(n):
        norm = np.sum(weights * p * p)
        a[k] = np.sum(weights * nodes * p * p) / norm
        b[k] = norm if k == 0 else norm / norm_prev
        p_next = (nodes - a[k]) * p - (b[k] if k > 0 else 0.0) * p_prev
        # the monic polynomials shrink or grow geometrically: rescale the
        # pair (p_k, p_{k+1}) by one factor, which leaves the coefficients
        sc = 1.0 / np.sqrt(norm)
        p_prev, p = p * sc, p_next * sc
        norm_prev = 1.0
    return a, b


def chain_coefficients(J, omega_c, n_modes, points=4000):
    """(t0, omega[0..n_modes), t[0..n_modes-1)) of the mapped chain."""
    nodes, weights = discretised_measure(J, omega_c, points)
    a, b = stieltjes(nodes, weights, n_modes + 1)
    return float(np.sqrt(b[0])), a[:n_modes].copy(), np.sqrt(b[1:n_modes])
