"""Exact single-particle propagation of the Trotterised XX chain.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

With the Jordan-Wigner map (|0> empty, |1> occupied, n_i = (1 - Z_i)/2),
(X_b X_{b+1} + Y_b Y_{b+1})/2 = c_b^dag c_{b+1} + c_{b+1}^dag c_b and
h_i Z_i = h_i (1 - 2 n_i).  Every bond term h_b of the XX-plus-field chain
(with the on-site split used by the TEBD gates) is therefore a quadratic form
c^dag m_b c plus a constant, and the gate exp(-i tau h_b) acts on the
annihilation operators as c -> exp(-i tau m_b) c.  A product of gates acts as
the product of these N x N matrices in the same order, and the correlation
matrix C_ij = <c_i^dag c_j> evolves as C -> U^* C U^T.  This gives <Z_i>
after the whole Trotter circuit exactly, with no truncation, for any N.
"""
import numpy as np
import scipy.linalg

from .models import onsite_weight
from .mps import STEP_SWEEPS


def bond_matrix(b, couplings, fields):
    """Single-particle matrix (N x N) of bond term h_b."""
    n = len(fields)
    m = np.zeros((n, n), dtype=np.complex128)
    m[b, b + 1] = couplings[b]
    m[b + 1, b] = couplings[b]
    m[b, b] += -2.0 * fields[b] * onsite_weight(b, n)
    m[b + 1, b + 1] += -2.0 * fields[b + 1] * onsite_weight(b + 1, n)
    return m


def trotter_propagator(couplings, fields, dt, steps):
    """U_total of the symmetric Trotter circuit in single-particle space."""
    n = len(fields)
    u = np.eye(n, dtype=np.complex128)
    gates = {}
    for _ in range(steps):
        for parity, frac in STEP_SWEEPS:
            tau = frac * dt
            for b in range(parity, n - 1, 2):
                key = (b, tau)
                if key not in gates:
                    gates[key] = scipy.linalg.expm(-1j * tau * bond_matrix(b, couplings, fields))
                u = gates[key] @ u
    return u


def z_profile(couplings, fields, occupations, dt, steps):
    """<Z_i> after the Trotter circuit from a basis state with given n_i."""
    u = trotter_propagator(couplings, fields, dt, steps)
    c0 = np.diag(np.asarray(occupations, dtype=np.float64)).astype(np.complex128)
    c = u.conj() @ c0 @ u.T
    return 1.0 - 2.0 * np.real(np.diag(c))


def z_gradient(couplings, fields, occupations, dt, steps, site=0, h=1e-3):
    """d<Z_site>/dJ_b of the closed form for every bond coupling J_b.

    Central differences at steps h and h/2 combined by Richardson
    extrapolation (error O(h^4)); the closed form is smooth in J.
    """
    couplings = np.asarray(couplings, dtype=np.float64)
    grad = np.zeros(len(couplings))
    for b in range(len(couplings)):
        def central(step):
            up = couplings.copy()
            up[b] += step
            dn = couplings.copy()
            dn[b] -= step
            return (z_profile(up, fields, occupations, dt, steps)[site]
                    - z_profile(dn, fields, occupations, dt, steps)[site]) / (2.0 * step)
        grad[b] = (4.0 * central(h / 2.0) - central(h)) / 3.0
    return grad
