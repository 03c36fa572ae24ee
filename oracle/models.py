"""Nearest-neighbour Hamiltonians and two-site Trotter gates (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A chain Hamiltonian H = sum_b h_b is written as a sum of bond terms h_b on
sites (b, b+1), the form TEBD needs (Sec. II).  On-site terms are split
between the two bonds that share a site, half to each; the first and last
sites belong to one bond only and give it their whole on-site term.  The
two-site gate is G_b(tau) = exp(-i tau h_b) (Schroedinger propagator; the
paper writes the exponent with the opposite sign in Eq. (defst3rd)), indexed
row (i_k, i_{k+1}) -> i_k * d_{k+1} + i_{k+1} (Kronecker order).

Models:
* transverse-field Ising: H = -J sum Z_b Z_{b+1} - h sum X_i;
* XX plus field: H = sum_b J_b (X_b X_{b+1} + Y_b Y_{b+1}) / 2 + sum_i h_i Z_i;
* chain-mapped spin-boson, Eq. (H_1D): site 0 a spin with
  H_sys = (omega0/2) sigma_z, coupled by t0 sigma_x (b_1 + b_1^dag) to the
  first oscillator; oscillators n >= 1 with omega_n b_n^dag b_n and hopping
  t_n (b_n^dag b_{n+1} + b_n b_{n+1}^dag); oscillators truncated to d levels
  (Sec. III, local-dimension truncation), b|n> = sqrt(n)|n-1>.

Spin basis: |0> has Z = +1 (spin up), |1> has Z = -1.
"""
import numpy as np
import scipy.linalg

X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def boson_annihilation(d):
    """Truncated bosonic b on levels 0..d-1: b|n> = sqrt(n)|n-1>."""
    b = np.zeros((d, d), dtype=np.complex128)
    for n in range(1, d):
        b[n - 1, n] = np.sqrt(n)
    return b


def onsite_weight(site, n_sites):
    """Share of a site's on-site term carried by each of its bonds."""
    if n_sites == 2:
        return 1.0
    return 1.0 if site in (0, n_sites - 1) else 0.5


def bond_hamiltonians(dims, two_site, onsite):
    """h_b = two_site[b] + w_b * onsite[b] x 1 + w_{b+1} * 1 x onsite[b+1]."""
    n = len(dims)
    out = []
    for b in range(n - 1):
        da, db = dims[b], dims[b + 1]
        h = np.array(two_site[b], dtype=np.complex128).copy()
        h += onsite_weight(b, n) * np.kron(onsite[b], np.eye(db))
        h += onsite_weight(b + 1, n) * np.kron(np.eye(da), onsite[b + 1])
        out.append(h)
    return out


def tfim(n_sites, J=1.0, h=1.0):
    """Bond terms of the open transverse-field Ising chain."""
    dims = [2] * n_sites
    two = [-J * np.kron(Z, Z) for _ in range(n_sites - 1)]
    ons = [-h * X for _ in range(n_sites)]
    return dims, bond_hamiltonians(dims, two, ons)


def xx_field(couplings, fields):
    """Bond terms of the XX chain with site-dependent couplings and Z fields."""
    n_sites = len(fields)
    dims = [2] * n_sites
    two = [Jb * 0.5 * (np.kron(X, X) + np.kron(Y, Y)) for Jb in couplings]
    ons = [hi * Z for hi in fields]
    return dims, bond_hamiltonians(dims, two, ons)


def spin_boson_chain(n_sites, d, omega0=1.0, t0=0.5, omegas=1.0, hops=0.5):
    """Bond terms of the chain-mapped spin-boson model, Eq. (H_1D)."""
    dims = [2] + [d] * (n_sites - 1)
    b = boson_annihilation(d)
    bd = b.conj().T
    ons = [0.5 * omega0 * Z] + [omegas * (bd @ b) for _ in range(n_sites - 1)]
    two = [t0 * np.kron(X, b + bd)]
    for _ in range(1, n_sites - 1):
        two.append(hops * (np.kron(bd, b) + np.kron(b, bd)))
    return dims, bond_hamiltonians(dims, two, ons)


def gate(h_bond, tau):
    """Two-site propagator G = exp(-i tau h_b) by scipy's Pade expm."""
    return scipy.linalg.expm(-1j * tau * np.asarray(h_bond, dtype=np.complex128))


def full_hamiltonian(dims, bond_hams):
    """Dense H = sum_b h_b on the whole chain (small systems only)."""
    total = int(np.prod(dims))
    H = np.zeros((total, total), dtype=np.complex128)
    for b, hb in enumerate(bond_hams):
        left = int(np.prod(dims[:b]))
        right = int(np.prod(dims[b + 2:]))
        H += np.kron(np.kron(np.eye(left), hb), np.eye(right))
    return H


def spin_boson_chain_general(dims, omega0, t0, omegas, hops):
    """Eq. (H_1D) with site-dependent frequencies omegas[k] and hoppings
    hops[k] (between oscillators k and k+1, 0-based over the oscillators)
    and oscillator truncations dims[1:] (TEDOPA chains, Sec. III)."""
    n = len(dims)
    bs = [boson_annihilation(d) for d in dims[1:]]
    ons = [0.5 * omega0 * Z] + [omegas[k] * (b.conj().T @ b) for k, b in enumerate(bs)]
    two = [t0 * np.kron(X, bs[0] + bs[0].conj().T)]
    for k in range(n - 2):
        two.append(hops[k] * (np.kron(bs[k].conj().T, bs[k + 1]) + np.kron(bs[k], bs[k + 1].conj().T)))
    return list(dims), bond_hamiltonians(list(dims), two, ons)
