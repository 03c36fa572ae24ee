"""Mixed-state TEBD: density matrices as MPOs in Liouville space (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper: Sec. II (mixed states): the density matrix is written as a matrix
product operator; the TEBD recipe stays the same with the local dimension
squared, two-site gates built for the density matrix, and normalisation and
measurements adapted.  Sec. V.B samples the Theta matrices of its timing
tables (Table II) from such simulations, of size d^2 chi x d^2 chi.

Conventions (the GPU path must use the same ones):
* Local index of site k: alpha = i * d_k + j for the operator |i><j|, so the
  MPO of a density matrix is an MPS with local dimensions d_k^2 whose
  coefficient of (alpha_0 ... alpha_{N-1}) is rho[(i_0..i_{N-1}), (j_0..j_{N-1})].
* A bond generator is the Lindblad map restricted to the two sites,
  L_b(rho) = -i [h_b, rho] + sum_c (c rho c^+ - (c^+ c rho + rho c^+ c) / 2),
  with each site's jump operators shared between its two bonds like the
  on-site Hamiltonian terms (weight 1/2 each, 1 for an end site: the
  dissipators of different sites commute, so the shares add up).  It is a
  (d_l^2 d_r^2) x (d_l^2 d_r^2) matrix in the two-site MPO index
  (alpha_l, alpha_r) -> alpha_l * d_r^2 + alpha_r; the gate of a sweep is
  exp(tau L_b).  Without jump operators the gate is U rho U^+ with
  U = exp(-i tau h_b).
* Observables: <O_k> = tr(O_k rho) / tr(rho), by contracting the MPO with
  the identity on every other site (the truncation renormalises the MPO in
  the Frobenius norm, Sec. II.C; the ratio does not see that scale).
"""
import numpy as np
import scipy.linalg

from . import models


def local_basis_vector(rho):
    """Row-major vectorisation of a local density matrix: entry i * d + j."""
    rho = np.asarray(rho, dtype=np.complex128)
    return rho.reshape(-1)


def bond_generator(h, dl, dr, jumps):
    """The two-site Lindblad generator as a matrix, by its definition.

    jumps: list of (d_l d_r) x (d_l d_r) jump operators (already carrying
    their share weights).  Column (alpha_l, alpha_r) is the image of the
    basis operator |i_l i_r><j_l j_r| written in the MPO index order.
    """
    h = np.asarray(h, dtype=np.complex128)
    D = dl * dr
    dim = D * D
    out = np.zeros((dim, dim), dtype=np.complex128)

    def to_mpo_index(il, jl, ir, jr):
        return (il * dl + jl) * (dr * dr) + (ir * dr + jr)

    for il in range(dl):
        for jl in range(dl):
            for ir in range(dr):
                for jr in range(dr):
                    e = np.zeros((D, D), dtype=np.complex128)
                    e[il * dr + ir, jl * dr + jr] = 1.0
                    img = -1j * (h @ e - e @ h)
                    for c in jumps:
                        cd = c.conj().T
                        img = img + c @ e @ cd - 0.5 * (cd @ c @ e + e @ cd @ c)
                    col = to_mpo_index(il, jl, ir, jr)
                    for a in range(D):
                        for b in range(D):
                            if img[a, b] != 0:
                                ail, air = divmod(a, dr)
                                bjl, bjr = divmod(b, dr)
                                out[to_mpo_index(ail, bjl, air, bjr), col] += img[a, b]
    return out


def bond_generators(dims, bond_hams, site_jumps):
    """Generators of every bond; site_jumps[k] lists the jump operators of
    site k (d_k x d_k), shared between its bonds like on-site terms."""
    n = len(dims)
    gens = []
    for b in range(n - 1):
        dl, dr = dims[b], dims[b + 1]
        jumps = []
        wl = models.onsite_weight(b, n)
        wr = models.onsite_weight(b + 1, n)
        for c in site_jumps[b]:
            jumps.append(np.sqrt(wl) * np.kron(c, np.eye(dr)))
        for c in site_jumps[b + 1]:
            jumps.append(np.sqrt(wr) * np.kron(np.eye(dl), c))
        gens.append(bond_generator(bond_hams[b], dl, dr, jumps))
    return gens


def gate(generator, tau):
    """exp(tau L) by scipy's matrix exponential."""
    return scipy.linalg.expm(tau * np.asarray(generator, dtype=np.complex128))


def trace_expectation(mps, op, site):
    """tr(O_site rho) / tr(rho) of an MPO held as an MPS over d^2 (Vidal
    form), by exact contraction with the identity on the other sites."""
    n = mps.n_sites
    env_o = np.ones(1, dtype=np.complex128)
    env_t = np.ones(1, dtype=np.complex128)
    for k in range(n):
        g = mps.gammas[k]
        d = int(round(np.sqrt(g.shape[0])))
        lam = mps.lambdas[k] if k < n - 1 else np.ones(1)
        a = g * lam[None, None, :]
        ident = np.eye(d, dtype=np.complex128).reshape(-1)
        # tr(O rho) = sum_ij O_ji rho_ij: weight of local index i*d+j is O[j, i]
        w_o = np.asarray(op, dtype=np.complex128).T.reshape(-1) if k == site else ident
        env_o = np.einsum("a,iac,i->c", env_o, a, w_o)
        env_t = np.einsum("a,iac,i->c", env_t, a, ident)
    return complex(env_o[0] / env_t[0])


def full_generator(dims, bond_gens):
    """Sum of the bond generators acting on the whole chain's vec(rho)
    (MPO index order), for exact evolution of small chains."""
    ldims = [d * d for d in dims]
    total = int(np.prod(ldims))
    out = np.zeros((total, total), dtype=np.complex128)
    for b, g in enumerate(bond_gens):
        left = int(np.prod(ldims[:b]))
        right = int(np.prod(ldims[b + 2:]))
        out += np.kron(np.kron(np.eye(left), g), np.eye(right))
    return out


def vec_trace_expectation(vec, op, site, dims):
    """tr(O_site rho) / tr(rho) of a full vec(rho) in MPO index order."""
    t = np.asarray(vec, dtype=np.complex128)
    num = t
    den = t
    for k in reversed(range(len(dims))):
        d = dims[k]
        ident = np.eye(d, dtype=np.complex128).reshape(-1)
        w = np.asarray(op, dtype=np.complex128).T.reshape(-1) if k == site else ident
        num = num.reshape(-1, d * d) @ w
        den = den.reshape(-1, d * d) @ ident
    return complex(num[0] / den[0])
