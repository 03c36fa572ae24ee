"""Host-side builders of chain Hamiltonians and two-site gates (inputs only).

The bond update takes the two-site gate as an input (Sec. II.B, Eq.
defupdatetheta); these helpers prepare it once, off the device path.
H = sum_b h_b with h_b on sites (b, b+1); each site's on-site term is shared
half and half by its two bonds (whole on the first and last site).  The gate
of a step tau is G_b = exp(-i tau h_b), computed from the eigendecomposition
of the Hermitian h_b, indexed (i_k, i_{k+1}) -> i_k * d_{k+1} + i_{k+1}.
Spin basis: |0> has sigma_z = +1.

Models: transverse-field Ising, XX chain with site fields, and the
chain-mapped spin-boson model of Sec. III, Eq. (H_1D), with oscillators
truncated to d levels.
"""
import numpy as np

PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def lowering(d):
    """b on d levels: b|n> = sqrt(n)|n-1>."""
    return np.diag(np.sqrt(np.arange(1, d, dtype=np.float64)), k=1).astype(np.complex128)


def _split(site, n_sites):
    if n_sites == 2 or site == 0 or site == n_sites - 1:
        return 1.0
    return 0.5


def _assemble(dims, pair_terms, site_terms):
    n = len(dims)
    hs = []
    for b in range(n - 1):
        dl, dr = dims[b], dims[b + 1]
        h = np.asarray(pair_terms[b], dtype=np.complex128)
        h = h + _split(b, n) * np.kron(site_terms[b], np.eye(dr))
        h = h + _split(b + 1, n) * np.kron(np.eye(dl), site_terms[b + 1])
        hs.append(h)
    return hs


def transverse_ising(n_sites, J=1.0, h=1.0):
    """H = -J sum Z Z - h sum X; returns (dims, bond Hamiltonians)."""
    dims = [2] * n_sites
    zz = np.kron(PAULI_Z, PAULI_Z)
    return dims, _assemble(dims, [-J * zz] * (n_sites - 1), [-h * PAULI_X] * n_sites)


def xx_chain(couplings, fields):
    """H = sum J_b (X X + Y Y)/2 + sum h_i Z_i."""
    n_sites = len(fields)
    dims = [2] * n_sites
    hop = 0.5 * (np.kron(PAULI_X, PAULI_X) + np.kron(PAULI_Y, PAULI_Y))
    return dims, _assemble(dims, [J * hop for J in couplings], [h * PAULI_Z for h in fields])


def spin_boson(n_sites, d, omega0=1.0, t0=0.5, omegas=1.0, hops=0.5):
    """Eq. (H_1D): (omega0/2) sigma_z + t0 sigma_x (b_1 + b_1^dag)
    + sum omega b^dag b + sum t (b_n^dag b_{n+1} + h.c.)."""
    dims = [2] + [d] * (n_sites - 1)
    b = lowering(d)
    bd = b.conj().T
    site = [0.5 * omega0 * PAULI_Z] + [omegas * bd @ b] * (n_sites - 1)
    pair = [t0 * np.kron(PAULI_X, b + bd)] + [hops * (np.kron(bd, b) + np.kron(b, bd))] * (n_sites - 2)
    return dims, _assemble(dims, pair, site)


def propagator(h, tau):
    """exp(-i tau h) for Hermitian h via its eigendecomposition."""
    h = np.asarray(h, dtype=np.complex128)
    e, v = np.linalg.eigh(0.5 * (h + h.conj().T))
    return (v * np.exp(-1j * tau * e)[None, :]) @ v.conj().T


def gate_stack(dims, bond_hams, tau):
    """Gates of every bond, padded to (N-1, d_max^2, d_max^2) (complex128)."""
    dmax = max(dims)
    out = np.zeros((len(bond_hams), dmax * dmax, dmax * dmax), dtype=np.complex128)
    for b, h in enumerate(bond_hams):
        g = propagator(h, tau)
        k = g.shape[0]
        out[b, :k, :k] = g
    return out


# ---------------------------------------------------------------------------
# Mixed states (Sec. II): the density matrix as an MPO, i.e. an MPS over the
# local operator space of dimension d^2 with local index i * d + j for
# |i><j|.  A bond's gate is exp(tau L_b) with the two-site Lindblad generator
# L_b(rho) = -i [h_b, rho] + sum_c (c rho c^+ - {c^+ c, rho} / 2), each
# site's jump operators shared between its bonds like its on-site terms.

def _lindblad_matrix(h, jumps):
    """Generator on the row-major vec(rho) of the two-site density matrix:
    A rho B -> (A kron B^T) vec(rho)."""
    D = h.shape[0]
    eye = np.eye(D, dtype=np.complex128)
    out = -1j * (np.kron(h, eye) - np.kron(eye, h.T))
    for c in jumps:
        cdc = c.conj().T @ c
        out = out + np.kron(c, c.conj()) - 0.5 * (np.kron(cdc, eye) + np.kron(eye, cdc.T))
    return out


def liouville_generators(dims, bond_hams, site_jumps):
    """Bond generators in the two-site MPO index (i_l d_l + j_l) d_r^2 +
    (i_r d_r + j_r); site_jumps[k]: jump operators (d_k x d_k) of site k."""
    n = len(dims)
    gens = []
    for b in range(n - 1):
        dl, dr = dims[b], dims[b + 1]
        jumps = [np.sqrt(_split(b, n)) * np.kron(c, np.eye(dr)) for c in site_jumps[b]]
        jumps += [np.sqrt(_split(b + 1, n)) * np.kron(np.eye(dl), c) for c in site_jumps[b + 1]]
        g = _lindblad_matrix(np.asarray(bond_hams[b], dtype=np.complex128), jumps)
        # (i_l, i_r, j_l, j_r) x (k_l, k_r, l_l, l_r) -> (i_l, j_l, i_r, j_r) x (k_l, l_l, k_r, l_r)
        g = g.reshape(dl, dr, dl, dr, dl, dr, dl, dr).transpose(0, 2, 1, 3, 4, 6, 5, 7)
        gens.append(np.ascontiguousarray(g.reshape(dl * dl * dr * dr, -1)))
    return gens


def generator_gate_stack(local_dims, generators, tau):
    """exp(tau L_b) of every bond (torch's matrix exponential on the host),
    padded to (N-1, D_max^2, D_max^2) with D the local (operator) dims."""
    import torch
    dmax = max(local_dims)
    out = np.zeros((len(generators), dmax * dmax, dmax * dmax), dtype=np.complex128)
    for b, g in enumerate(generators):
        e = torch.linalg.matrix_exp(torch.from_numpy(tau * np.asarray(g, dtype=np.complex128)))
        k = e.shape[0]
        out[b, :k, :k] = e.numpy()
    return out


def spin_boson_tedopa(dims, t0, omegas, hops, omega0=1.0):
    """Eq. (H_1D) with site-dependent chain coefficients (from
    tedopa.chain_coefficients) and oscillator truncations dims[1:]:
    (omega0/2) sigma_z + t0 sigma_x (b_1 + b_1^dag) + sum_n omega_n b_n^dag b_n
    + sum_n t_n (b_n^dag b_{n+1} + h.c.)."""
    n = len(dims)
    ops = [lowering(d) for d in dims[1:]]
    site = [0.5 * omega0 * PAULI_Z] + [omegas[k] * b.conj().T @ b for k, b in enumerate(ops)]
    pair = [t0 * np.kron(PAULI_X, ops[0] + ops[0].conj().T)]
    for k in range(n - 2):
        bl, br = ops[k], ops[k + 1]
        pair.append(hops[k] * (np.kron(bl.conj().T, br) + np.kron(bl, br.conj().T)))
    return list(dims), _assemble(list(dims), pair, site)
