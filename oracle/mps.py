"""Vidal-form MPS, the two-site bond update and the TEBD sweep (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper: Tamascelli, Rosenbach, Plenio, arXiv:1504.00992, Sec. II.

State (Eq. defmps / relcoefmat): site k carries d_k matrices Gamma^[k]i of
size chi_k x chi_{k+1}; bond b (between sites b and b+1) carries the
diagonal lambda^[b] of length chi_{b+1}; chi_0 = chi_N = 1.  Arrays here:
gammas[k] has shape (d_k, chi_k, chi_{k+1}); lambdas[b] has shape
(chi_{b+1},).  Outside the chain lambda is taken as [1].

Bond update on bond b (sites k = b, k+1):
  Theta(i, j, a, c) = sum_g lam_l[a] Gk[i, a, g] lam_m[g] Gk1[j, g, c] lam_r[c]   Eq. (deftheta)
  Theta~(i, j, a, c) = sum_{i'j'} G[(i j), (i' j')] Theta(i', j', a, c)           Eq. (defupdatetheta)
  A[(i, a), (j, c)] = Theta~(i, j, a, c), row i*chi_l + a, col j*chi_r + c          (blocked form, Sec. II.B)
  A ~= U diag(s) V^H truncated to chi' (full SVD or RRSVD), lambda' = s / ||s||
  Gamma'^[k]  [i, a, g] = U[(i, a), g] / lam_l[a]
  Gamma'^[k+1][j, g, c] = V^H[g, (j, c)] / lam_r[c]
The division uses 1/lam only above a floor (default 1e-14) and 0 below it;
the paper only says the new Gamma must be extracted from the factors.
"""
import numpy as np

from . import rrsvd as rr
from .philox import gaussian_omega

STATUS_LAMBDA_FLOOR = 8


class MPS:
    """Plain container: lists of Gamma tensors and lambda vectors."""

    def __init__(self, gammas, lambdas):
        self.gammas = [np.asarray(g, dtype=np.complex128) for g in gammas]
        self.lambdas = [np.asarray(l, dtype=np.float64) for l in lambdas]

    @property
    def n_sites(self):
        return len(self.gammas)

    @property
    def dims(self):
        return [g.shape[0] for g in self.gammas]

    def chis(self):
        """chi_0..chi_N (length N+1)."""
        return [1] + [len(l) for l in self.lambdas] + [1]

    def copy(self):
        return MPS([g.copy() for g in self.gammas], [l.copy() for l in self.lambdas])


def product_state(local_vectors):
    """MPS of a product state; each site's vector is normalised."""
    gammas = []
    for v in local_vectors:
        v = np.asarray(v, dtype=np.complex128)
        v = v / np.linalg.norm(v)
        gammas.append(v.reshape(-1, 1, 1))
    lambdas = [np.ones(1) for _ in range(len(local_vectors) - 1)]
    return MPS(gammas, lambdas)


def basis_product_state(dims, levels):
    """Product of computational basis states |levels[k]> on sites of dims."""
    vecs = []
    for d, lv in zip(dims, levels):
        v = np.zeros(d, dtype=np.complex128)
        v[lv] = 1.0
        vecs.append(v)
    return product_state(vecs)


def outer_lambdas(mps, b):
    """lambda to the left of site b and to the right of site b+1."""
    n = mps.n_sites
    lam_l = mps.lambdas[b - 1] if b >= 1 else np.ones(1)
    lam_r = mps.lambdas[b + 1] if b + 1 <= n - 2 else np.ones(1)
    return lam_l, lam_r


def theta(mps, b):
    """Eq. (deftheta): Theta(i, j, a, c) for bond b."""
    lam_l, lam_r = outer_lambdas(mps, b)
    lam_m = mps.lambdas[b]
    gk = mps.gammas[b]
    gk1 = mps.gammas[b + 1]
    return np.einsum("a,iag,g,jgc,c->ijac", lam_l, gk, lam_m, gk1, lam_r)


def apply_gate(gate, th):
    """Eq. (defupdatetheta): mix the physical index pair with the gate."""
    di, dj, cl, cr = th.shape
    g4 = np.asarray(gate, dtype=np.complex128).reshape(di, dj, di, dj)
    return np.einsum("ijxy,xyac->ijac", g4, th)


def blocked(th):
    """Blocked matrix A[(i, a), (j, c)] of Sec. II.B."""
    di, dj, cl, cr = th.shape
    return th.transpose(0, 2, 1, 3).reshape(di * cl, dj * cr)


def safe_inverse(lam, floor):
    """1/lam where lam > floor, 0 elsewhere; also whether the floor was hit."""
    lam = np.asarray(lam, dtype=np.float64)
    inv = np.zeros_like(lam)
    big = lam > floor
    inv[big] = 1.0 / lam[big]
    return inv, bool(np.any(~big))


def bond_update(mps, b, gate, chi_max, eps, method="full", omega=None, q=2,
                lambda_floor=1e-14, p=10):
    """Apply the gate to bond b and truncate; updates mps in place.

    method "full": O-def (LAPACK SVD of the blocked Theta~).
    method "rrsvd": O-alg with the given Omega and q power iterations.
    method "rrsvd_adaptive": two-stage adaptive rank; `omega` is then a
    function l -> n x l test matrix, the first-stage rank follows the bond
    dimension before the update (rrsvd.first_stage_rank).
    method "rrsvd_accuracy": the Accuracy Check of Sec. IV (Alg. 2) from
    k0 = the bond dimension before the update, probes of r = p columns;
    `omega` is then a function (c0, w) -> columns c0 .. c0 + w - 1 of the
    bond's Gaussian stream.
    Returns a dict with chi', discarded weight w, status bits, and the
    singular values before renormalisation.
    """
    lam_l, lam_r = outer_lambdas(mps, b)
    th = apply_gate(gate, theta(mps, b))
    di, dj, cl, cr = th.shape
    a = blocked(th)
    if method == "full":
        u, s, vh, chi, w, status = rr.truncate_full_svd(a, chi_max, eps)
    elif method == "rrsvd":
        u, s, vh, chi, w, status = rr.truncate_rrsvd(a, omega, q, chi_max, eps)
    elif method == "rrsvd_adaptive":
        k1 = rr.first_stage_rank(len(mps.lambdas[b]), chi_max)
        u, s, vh, chi, w, status, stage = rr.truncate_rrsvd_adaptive(a, omega, q, chi_max, eps, k1, p)
    elif method == "rrsvd_accuracy":
        # start from the bond dimension before the update; probes of p columns
        u, s, vh, chi, w, status, rounds = rr.truncate_rrsvd_accuracy(
            a, omega, q, chi_max, eps, len(mps.lambdas[b]), p, p)
    else:
        raise ValueError(method)
    norm = np.sqrt(np.sum(s ** 2))
    lam_new = s / norm if norm > 0 else s
    inv_l, hit_l = safe_inverse(lam_l, lambda_floor)
    inv_r, hit_r = safe_inverse(lam_r, lambda_floor)
    if hit_l or hit_r:
        status |= STATUS_LAMBDA_FLOOR
    gk = u.reshape(di, cl, chi) * inv_l[None, :, None]
    gk1 = vh.reshape(chi, dj, cr).transpose(1, 0, 2) * inv_r[None, None, :]
    mps.gammas[b] = gk
    mps.gammas[b + 1] = gk1
    mps.lambdas[b] = lam_new
    return {"chi": chi, "w": w, "status": status, "s": s, "frob2": float(np.vdot(a, a).real)}


# Sweep order of one time step, Eq. (defst3rd): F/2 (even bonds, tau = dt/2),
# G (odd bonds, tau = dt), F/2 again; three sweeps, none merged.
STEP_SWEEPS = ((0, 0.5), (1, 1.0), (0, 0.5))


def step_sweeps(order=2):
    """(parity, tau / dt) of every sweep of one time step.

    order 2: Eq. (defst3rd).  order 4: the paper's higher-order schemes
    (Sec. II.C) in Suzuki's fractal form: the symmetric step S(x) of
    Eq. (defst3rd) composed as S(s dt) S(s dt) S((1 - 4 s) dt) S(s dt)
    S(s dt) with s = 1 / (4 - 4^(1/3)), which cancels the third-order error
    of the symmetric product (local error O(dt^5)).  Fifteen sweeps; the
    half sweeps where two S meet are kept separate, as in order 2.
    """
    if order == 2:
        return STEP_SWEEPS
    if order == 4:
        s = 1.0 / (4.0 - 4.0 ** (1.0 / 3.0))
        out = []
        for x in (s, s, 1.0 - 4.0 * s, s, s):
            out += [(0, 0.5 * x), (1, x), (0, 0.5 * x)]
        return tuple(out)
    raise ValueError("order must be 2 or 4")


class TEBD:
    """Plain TEBD driver over one chain.

    gate_fn(b, tau) returns the two-site gate of bond b for step tau.
    RRSVD problems draw Omega from Philox with problem id
    chain * (N - 1) + b and call id = the running sweep counter.
    """

    def __init__(self, mps, gate_fn, dt, chi_max, eps, method="full", p=10, q=2,
                 seed=0, chain=0, lambda_floor=1e-14, order=2):
        self.mps = mps
        self.sweeps = step_sweeps(order)
        self.gate_fn = gate_fn
        self.dt = dt
        self.chi_max = chi_max
        self.eps = eps
        self.method = method
        self.p = p
        self.q = q
        self.seed = seed
        self.chain = chain
        self.lambda_floor = lambda_floor
        self.sweeps_done = 0
        self.log = []

    def sweep(self, parity, tau):
        n = self.mps.n_sites
        for b in range(parity, n - 1, 2):
            omega = None
            chis = self.mps.chis()
            dims = self.mps.dims
            ncol = dims[b + 1] * chis[b + 2]
            pid = self.chain * (n - 1) + b
            if self.method == "rrsvd":
                m = dims[b] * chis[b]
                l = rr.sketch_width(self.chi_max, self.p, m, ncol)
                omega = gaussian_omega(ncol, l, self.seed, pid, self.sweeps_done)
            elif self.method == "rrsvd_adaptive":
                sweep_id = self.sweeps_done

                def omega(l, ncol=ncol, pid=pid, sweep_id=sweep_id):
                    return gaussian_omega(ncol, l, self.seed, pid, sweep_id)
            elif self.method == "rrsvd_accuracy":
                sweep_id = self.sweeps_done

                def omega(c0, w, ncol=ncol, pid=pid, sweep_id=sweep_id):
                    return gaussian_omega(ncol, c0 + w, self.seed, pid, sweep_id)[:, c0:]
            info = bond_update(self.mps, b, self.gate_fn(b, tau), self.chi_max, self.eps,
                               self.method, omega, self.q, self.lambda_floor, self.p)
            info["bond"] = b
            info["sweep"] = self.sweeps_done
            self.log.append(info)
        self.sweeps_done += 1

    def step(self):
        for parity, frac in self.sweeps:
            self.sweep(parity, frac * self.dt)


def to_statevector(mps):
    """Contract the MPS into the full coefficient vector (Eq. relcoefmat)."""
    psi = mps.gammas[0][:, 0, :]  # (d0, chi1)
    for k in range(1, mps.n_sites):
        psi = psi * mps.lambdas[k - 1][None, :]
        g = mps.gammas[k]  # (dk, chi_k, chi_k+1)
        psi = np.einsum("pa,iac->pic", psi, g).reshape(-1, g.shape[2])
    return psi[:, 0]


def expectation(mps, op, site):
    """<psi|O_site|psi> / <psi|psi> by exact transfer-matrix contraction.

    Uses the plain matrices A^[k]i = Gamma^[k]i lambda^[k] (lambda^[N-1] = 1)
    and no canonical-form shortcut, so it is exact for any Gamma, lambda.
    """
    n = mps.n_sites
    env_o = np.ones((1, 1), dtype=np.complex128)
    env_n = np.ones((1, 1), dtype=np.complex128)
    for k in range(n):
        g = mps.gammas[k]
        lam = mps.lambdas[k] if k < n - 1 else np.ones(1)
        a = g * lam[None, None, :]
        opk = op if k == site else np.eye(g.shape[0])
        env_o = np.einsum("ab,iac,ij,jbd->cd", env_o, a.conj(), opk, a)
        env_n = np.einsum("ab,iac,ibd->cd", env_n, a.conj(), a)
    return complex(env_o[0, 0] / env_n[0, 0])


def norm2(mps):
    """<psi|psi> by exact contraction."""
    n = mps.n_sites
    env = np.ones((1, 1), dtype=np.complex128)
    for k in range(n):
        lam = mps.lambdas[k] if k < n - 1 else np.ones(1)
        a = mps.gammas[k] * lam[None, None, :]
        env = np.einsum("ab,iac,ibd->cd", env, a.conj(), a)
    return float(env[0, 0].real)


def local_expectation_canonical(mps, op, site):
    """Canonical-form formula sum |lam_l Gamma lam_r|^2 weighted by O.

    Exact only when the MPS is in Vidal canonical form; logged beside the
    exact contraction as a cross-check.
    """
    n = mps.n_sites
    lam_l = mps.lambdas[site - 1] if site >= 1 else np.ones(1)
    lam_r = mps.lambdas[site] if site <= n - 2 else np.ones(1)
    t = lam_l[None, :, None] * mps.gammas[site] * lam_r[None, None, :]
    return complex(np.einsum("iac,ij,jac->", t.conj(), op, t))
