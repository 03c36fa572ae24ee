"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method (no Theta contraction, no
gate, no sketch, QR, SVD or truncation).  It only draws inputs: matrices with
a prescribed spectrum, random Vidal-form tensors, couplings and fields, and
the initial product states of the benchmark chains.  Both the CPU oracle and
the HIP path consume the same draws.

Workloads (paper: Tamascelli, Rosenbach, Plenio, arXiv:1504.00992):
* known-spectrum matrices A = U diag(s) V^H with Haar U, V -- the paper's own
  construction for its stability tests (Sec. V.A);
* the batched standalone RRSVD set: 256 square matrices of sizes drawn
  uniformly from {256, 512, 1024, 2048}, s_i = exp(-i/25), i = 0..n-1;
* TFIM, XX-plus-random-field and chain-mapped spin-boson parameters.
"""
import numpy as np

BASE_SEED = 1504


def rng(seed):
    return np.random.default_rng(int(seed))


def ginibre(m, n, gen):
    """m x n complex Gaussian matrix, entries CN(0, 1)."""
    return (gen.standard_normal((m, n)) + 1j * gen.standard_normal((m, n))) / np.sqrt(2.0)


def haar_isometry(m, n, gen):
    """m x n matrix with Haar-distributed orthonormal columns (m >= n).

    QR of a complex Ginibre matrix with the phases of R's diagonal moved
    into Q (Mezzadri, Notices AMS 54 (2007) 592).
    """
    z = ginibre(m, n, gen)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def known_spectrum(m, n, s, gen):
    """A = U diag(s) V^H with Haar U (m x r), V (n x r), r = len(s)."""
    s = np.asarray(s, dtype=np.float64)
    r = len(s)
    u = haar_isometry(m, r, gen)
    v = haar_isometry(n, r, gen)
    return (u * s[None, :]) @ v.conj().T


def exp_spectrum(n, scale=25.0):
    """s_i = exp(-i / scale), i = 0..n-1."""
    return np.exp(-np.arange(n) / scale)


def batched_rrsvd_sizes(count=256, choices=(256, 512, 1024, 2048), seed=BASE_SEED):
    """Sizes of the batched standalone RRSVD workload (drawn uniformly)."""
    return [int(x) for x in rng(seed).choice(np.asarray(choices), size=count)]


def batched_rrsvd_matrix(n, index, seed=BASE_SEED):
    """Square matrix `index` of the batched workload: Haar x exp spectrum."""
    gen = rng(seed * 100003 + index)
    return known_spectrum(n, n, exp_spectrum(n), gen)


def batched_rrsvd_matrices_device(sizes, seed=BASE_SEED, device="cuda"):
    """The batched workload drawn on the device (same construction, faster).

    Haar factors from torch's QR of complex Ginibre matrices with the phase
    fix, spectrum s_i = exp(-i/25).  Returns a list of complex128 tensors.
    """
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = []
    for n in sizes:
        fac = []
        for _ in range(2):
            z = torch.randn((n, n), dtype=torch.complex128, device=device, generator=gen)
            q, r = torch.linalg.qr(z)
            d = torch.diagonal(r)
            fac.append(q * (d / d.abs())[None, :])
        s = torch.exp(-torch.arange(n, dtype=torch.float64, device=device) / 25.0)
        vh = fac[1].conj().transpose(0, 1).contiguous()
        out.append(((fac[0] * s[None, :]) @ vh).contiguous())
    return out


def random_vidal_bond(dl, dr, chi_l, chi_m, chi_r, gen, decay=0.3):
    """Random tensors around one bond: Gamma_k, Gamma_k+1 and three lambdas.

    The lambdas are positive, decreasing and unit-norm (exp(-decay*i)); the
    Gammas are complex Gaussian.  Theta built from them is a generic dense
    complex matrix of the bond-update shape.
    """
    def lam(c):
        v = np.exp(-decay * np.arange(c))
        return v / np.linalg.norm(v)
    gk = ginibre(dl * chi_l, chi_m, gen).reshape(dl, chi_l, chi_m)
    gk1 = ginibre(dr * chi_m, chi_r, gen).reshape(dr, chi_m, chi_r)
    return gk, gk1, lam(chi_l), lam(chi_m), lam(chi_r)


def random_vidal_chain(dims, chis, gen, decay=0.3):
    """Random Gammas and lambdas of one chain with bond dimensions chis.

    chis has length N + 1 with chis[0] = chis[N] = 1.  Gammas are complex
    Gaussian of shape (d_k, chi_k, chi_k+1); each lambda is positive,
    decreasing and unit-norm (exp(-decay * i)).  No canonical form.
    """
    gammas = [ginibre(d * chis[k], chis[k + 1], gen).reshape(d, chis[k], chis[k + 1])
              for k, d in enumerate(dims)]
    lambdas = []
    for b in range(len(dims) - 1):
        v = np.exp(-decay * np.arange(chis[b + 1]))
        lambdas.append(v / np.linalg.norm(v))
    return gammas, lambdas


def random_unitary(n, gen):
    """n x n Haar unitary (used as a generic two-site gate)."""
    return haar_isometry(n, n, gen)


def xx_couplings(n_sites, seed=BASE_SEED):
    """J_b ~ U[0.8, 1.2] (bonds) and h_i ~ U[-1, 1] (sites), seeded."""
    gen = rng(seed)
    J = gen.uniform(0.8, 1.2, size=n_sites - 1)
    h = gen.uniform(-1.0, 1.0, size=n_sites)
    return J, h


def neel_levels(n_sites):
    """|0101...>: site i in level i % 2."""
    return [i % 2 for i in range(n_sites)]


# Benchmark chain parameters.
TFIM_CFG = dict(n_sites=20, J=1.0, h=1.0, dt=0.01, steps=100, chi_max=32, p=10, q=2, eps=1e-10)
SPIN_BOSON_CFG = dict(n_sites=100, d=10, omega0=1.0, t0=0.5, omegas=1.0, hops=0.5, dt=0.05,
                      steps=200, chi_max=100, p=10, q=2, eps=1e-10, n_chains=16)
XX_CFG = dict(n_sites=40, chi_max=64, dt=0.02, steps=50, p=10, q=2, eps=1e-10, checkpoint=10)
