"""Brute-force state vectors: the same Trotter circuit, and exact evolution.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

These pin the MPS code: with no truncation, TEBD applies exactly the gates
of the Suzuki-Trotter circuit (Sec. II.C, Eq. defst3rd), so its state must
equal the state vector obtained by applying the same gates to the full
coefficient vector.  Exact diagonalisation gives exp(-iHt) itself, whose
distance to the circuit shrinks as dt^2 (second-order splitting).
"""
import numpy as np

from . import models
from .mps import step_sweeps


def product_vector(dims, levels):
    """Full coefficient vector of the basis product state |levels>."""
    psi = np.ones(1, dtype=np.complex128)
    for d, lv in zip(dims, levels):
        v = np.zeros(d, dtype=np.complex128)
        v[lv] = 1.0
        psi = np.kron(psi, v)
    return psi


def apply_two_site(psi, gate, b, dims):
    """Apply a (d_b d_{b+1}) x (d_b d_{b+1}) gate to sites b, b+1."""
    left = int(np.prod(dims[:b]))
    right = int(np.prod(dims[b + 2:]))
    dd = dims[b] * dims[b + 1]
    t = psi.reshape(left, dd, right)
    return np.einsum("xy,lyr->lxr", gate, t).reshape(-1)


def trotter_evolve(psi, bond_hams, dims, dt, steps, order=2):
    """Apply `steps` Trotter steps gate by gate (same order as TEBD)."""
    n = len(dims)
    for _ in range(steps):
        for parity, frac in step_sweeps(order):
            tau = frac * dt
            for b in range(parity, n - 1, 2):
                psi = apply_two_site(psi, models.gate(bond_hams[b], tau), b, dims)
    return psi


def exact_evolve(psi, H, t):
    """exp(-i H t) psi by diagonalising the Hermitian H."""
    e, v = np.linalg.eigh(H)
    return v @ (np.exp(-1j * e * t) * (v.conj().T @ psi))


def local_expectation(psi, op, site, dims):
    """<psi| O_site |psi> / <psi|psi>."""
    left = int(np.prod(dims[:site]))
    right = int(np.prod(dims[site + 1:]))
    t = psi.reshape(left, dims[site], right)
    val = np.einsum("lir,ij,ljr->", t.conj(), op, t)
    return complex(val / np.vdot(psi, psi))


def schmidt_values(psi, cut, dims):
    """Singular values of the coefficient matrix split after site `cut`."""
    left = int(np.prod(dims[:cut + 1]))
    return np.linalg.svd(psi.reshape(left, -1), compute_uv=False)
