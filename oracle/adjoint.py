"""Reverse-mode derivative of the TEBD bond update and of a whole TEBD run.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper does not differentiate its method.  This module states what the
derivative of the bond update of Sec. II computes (Theta of Eq. deftheta,
the gate of Eq. defupdatetheta, the truncated SVD of the blocked matrix,
renormalisation of the kept spectrum and lambda^-1 reabsorption), and gives
the references that a gradient of an observable with respect to Hamiltonian
couplings is checked against:

* ``tebd_gradient``: reverse mode over a recorded run, each bond undone by
  ``bond_adjoint``.  With the full LAPACK SVD (O-def) and every triplet
  coupled this is the exact derivative of the truncated map; with the RRSVD
  of Sec. IV (O-alg) it couples the kept triplets to the other triplets
  the sketch computed;
* ``finite_difference_gradient``: central differences of the O-def run with
  the bond dimensions of the base run replayed (truncation is piecewise);
* the free-fermion closed form of the Trotterised XX chain
  (``freefermion``), which carries no truncation at all.

Cotangent convention: for a real loss L and complex z = x + i y the
cotangent is zbar = dL/dx + i dL/dy, so that dL = Re sum conj(zbar) dz; a real
variable's cotangent is its plain derivative.  For a linear map Y = G X this
gives Xbar = G^H Ybar and Gbar = Ybar X^H.
"""
import numpy as np
import scipy.linalg

from . import mps as om
from . import rrsvd as rr
from .philox import gaussian_omega

ETA_REL = 1e-12


def broadened_gaps(s, eta):
    """F_ij = D / (D^2 + eta^2) with D = s_j^2 - s_i^2, and F_ii = 0.

    Away from degeneracies this is 1 / (s_j^2 - s_i^2); the broadening keeps
    it finite when two singular values coincide.
    """
    s2 = np.asarray(s, dtype=np.float64) ** 2
    d = s2[None, :] - s2[:, None]
    f = d / (d * d + eta * eta)
    np.fill_diagonal(f, 0.0)
    return f


def svd_backward(u, s, vh, ubar, sbar, vhbar, eta_rel=ETA_REL):
    """Cotangent of A for the triplets A ~= U diag(s) V^H (r of them).

    Abar = U [(J + J^H) S + S (K + K^H) + 1/2 S^-1 (L^H - L) + diag(sbar)] V^H
           + (I - U U^H) Ubar S^-1 V^H + U S^-1 Vbar^H (I - V V^H)
    with J = F o (U^H Ubar), K = F o (V^H Vbar), L = I o (V^H Vbar) and F from
    ``broadened_gaps`` with eta = eta_rel * s_1^2; 1/s_i is taken as 0 for
    s_i = 0.  The two projector terms are the limit of the coupling to the
    spectrum outside the r triplets when it vanishes.  Triplets that were
    computed but not kept enter with zero cotangents.  The loss must not
    depend on the phase of a singular pair.
    """
    u = np.asarray(u, dtype=np.complex128)
    vh = np.asarray(vh, dtype=np.complex128)
    s = np.asarray(s, dtype=np.float64)
    v = vh.conj().T
    vbar = np.asarray(vhbar, dtype=np.complex128).conj().T
    ubar = np.asarray(ubar, dtype=np.complex128)
    f = broadened_gaps(s, eta_rel * s[0] ** 2)
    sinv = np.zeros_like(s)
    sinv[s > 0] = 1.0 / s[s > 0]
    uhu = u.conj().T @ ubar
    vhv = v.conj().T @ vbar
    jm = f * uhu
    km = f * vhv
    lm = np.diag(np.diag(vhv))
    core = ((jm + jm.conj().T) @ np.diag(s) + np.diag(s) @ (km + km.conj().T)
            + 0.5 * np.diag(sinv) @ (lm.conj().T - lm) + np.diag(sbar))
    abar = u @ core @ vh
    abar = abar + (ubar - u @ uhu) @ np.diag(sinv) @ vh
    abar = abar + u @ np.diag(sinv) @ (vbar - v @ vhv).conj().T
    return abar


def bond_adjoint(gk, gk1, lam_l, lam_m, lam_r, gate, u, s, vh, chi, gk_bar_new, gk1_bar_new,
                 lam_bar_new, lambda_floor=1e-14, eta_rel=ETA_REL):
    """Undo one bond update (``mps.bond_update``) in reverse mode.

    Inputs: the tensors the update read (Gamma_k, Gamma_k+1, lambda_l,
    lambda_m, lambda_r, gate); the triplets U, s, V^H it computed, of which
    the first chi were kept (s before renormalisation); and the cotangents
    of what it wrote (Gamma'_k, Gamma'_k+1, lambda').
    Returns a dict with the cotangents of Gamma_k, Gamma_k+1 and lambda_m
    (which the update overwrote), the contributions to the cotangents of
    lambda_l and lambda_r (which it only read), and gate_bar.
    """
    di, cl, _ = gk.shape
    dj, _, cr = gk1.shape
    r = len(s)
    inv_l, _ = om.safe_inverse(lam_l, lambda_floor)
    inv_r, _ = om.safe_inverse(lam_r, lambda_floor)
    # lambda^-1 reabsorption of the kept columns:
    # Gamma'_k = U / lambda_l, Gamma'_k+1 = V^H / lambda_r
    gk_new = u[:, :chi].reshape(di, cl, chi) * inv_l[None, :, None]
    gk1_new = vh[:chi].reshape(chi, dj, cr).transpose(1, 0, 2) * inv_r[None, None, :]
    ubar = np.zeros((di * cl, r), dtype=np.complex128)
    ubar[:, :chi] = (gk_bar_new * inv_l[None, :, None]).reshape(di * cl, chi)
    vhbar = np.zeros((r, dj * cr), dtype=np.complex128)
    vhbar[:chi] = (gk1_bar_new * inv_r[None, None, :]).transpose(1, 0, 2).reshape(chi, dj * cr)
    lam_l_bar = -inv_l * np.einsum("iag,iag->a", gk_bar_new.conj(), gk_new).real
    lam_r_bar = -inv_r * np.einsum("jgc,jgc->c", gk1_bar_new.conj(), gk1_new).real
    # renormalisation lambda' = s_kept / ||s_kept||
    sk = s[:chi]
    nrm = np.sqrt(np.sum(sk ** 2))
    lam_new = sk / nrm
    sbar = np.zeros(r)
    sbar[:chi] = (lam_bar_new - lam_new * np.dot(lam_new, lam_bar_new)) / nrm
    abar = svd_backward(u, s, vh, ubar, sbar, vhbar, eta_rel)
    # blocked matrix A[(i, a), (j, c)] = Theta~(i, j, a, c)
    ttbar = abar.reshape(di, cl, dj, cr).transpose(0, 2, 1, 3)
    th = np.einsum("a,iag,g,jgc,c->ijac", lam_l, gk, lam_m, gk1, lam_r)
    g4 = np.asarray(gate, dtype=np.complex128).reshape(di, dj, di, dj)
    thbar = np.einsum("ijxy,ijac->xyac", g4.conj(), ttbar)
    gate_bar = np.einsum("ijac,xyac->ijxy", ttbar, th.conj()).reshape(di * dj, di * dj)
    # Theta(i, j, a, c) = lambda_l[a] Gk[i, a, g] lambda_m[g] Gk1[j, g, c] lambda_r[c]
    gk_bar = np.einsum("ijac,a,g,jgc,c->iag", thbar, lam_l, lam_m, gk1.conj(), lam_r)
    gk1_bar = np.einsum("ijac,a,iag,g,c->jgc", thbar, lam_l, gk.conj(), lam_m, lam_r)
    tc = thbar.conj()
    lam_l_bar = lam_l_bar + np.einsum("ijac,iag,g,jgc,c->a", tc, gk, lam_m, gk1, lam_r).real
    lam_m_bar = np.einsum("ijac,a,iag,jgc,c->g", tc, lam_l, gk, gk1, lam_r).real
    lam_r_bar = lam_r_bar + np.einsum("ijac,a,iag,g,jgc->c", tc, lam_l, gk, lam_m, gk1).real
    return {"gk_bar": gk_bar, "gk1_bar": gk1_bar, "lam_m_bar": lam_m_bar,
            "lam_l_bar": lam_l_bar, "lam_r_bar": lam_r_bar, "gate_bar": gate_bar}


def recorded_bond_update(mps, b, gate, chi_max, eps, method="full", omega_of=None, q=2, p=10,
                         chi_fixed=None, lambda_floor=1e-14):
    """Bond update that also returns what its adjoint needs.

    method "full": O-def, the same arithmetic as ``mps.bond_update``; every
    triplet of the LAPACK SVD is recorded; chi_fixed forces the kept rank
    (replay of a recorded schedule).  method "rrsvd": O-alg at the fixed
    sketch width min(chi_max + p, m, n); method "rrsvd_adaptive": O-alg with
    the two-stage rank (``rrsvd.adaptive_factors``).  The RRSVD methods
    record every triplet the accepted sketch gave.
    """
    lam_l, lam_r = om.outer_lambdas(mps, b)
    rec = {"b": b, "gk": mps.gammas[b].copy(), "gk1": mps.gammas[b + 1].copy(),
           "lam_l": lam_l.copy(), "lam_m": mps.lambdas[b].copy(), "lam_r": lam_r.copy(),
           "gate": np.asarray(gate, dtype=np.complex128)}
    th = om.apply_gate(gate, om.theta(mps, b))
    di, dj, cl, cr = th.shape
    a = om.blocked(th)
    if method == "full":
        u, s, vh = rr.lapack_svd(a)
        if chi_fixed is None:
            chi, _, _ = rr.truncation_rank(rr.tail_weights(s), chi_max, eps)
        else:
            chi = int(chi_fixed)
    elif method == "rrsvd":
        u, s, vh = rr.rrsvd(a, omega_of(rr.sketch_width(chi_max, p, *a.shape)), q)
        chi, _, _ = rr.truncation_rank(rr.frobenius_weights(s, float(np.vdot(a, a).real)),
                                       chi_max, eps)
    elif method == "rrsvd_adaptive":
        k1 = rr.first_stage_rank(len(mps.lambdas[b]), chi_max)
        u, s, vh, chi, _, _, _ = rr.adaptive_factors(a, omega_of, q, chi_max, eps, k1, p)
    else:
        raise ValueError(method)
    inv_l, _ = om.safe_inverse(lam_l, lambda_floor)
    inv_r, _ = om.safe_inverse(lam_r, lambda_floor)
    mps.gammas[b] = u[:, :chi].reshape(di, cl, chi) * inv_l[None, :, None]
    mps.gammas[b + 1] = vh[:chi].reshape(chi, dj, cr).transpose(1, 0, 2) * inv_r[None, None, :]
    mps.lambdas[b] = s[:chi] / np.sqrt(np.sum(s[:chi] ** 2))
    rec.update(u=u, s=s, vh=vh, chi=chi)
    return rec


def run_recorded(mps0, gate_fn, dt, steps, chi_max, eps, method="full", q=2, p=10, seed=0,
                 chain=0, schedule=None, lambda_floor=1e-14):
    """Forward TEBD (sweep order of ``mps.STEP_SWEEPS``) recording every update.

    gate_fn(b, tau) gives the gate.  RRSVD problems draw Omega as
    ``mps.TEBD`` does (problem id chain * (N - 1) + b, call id the sweep
    counter).  schedule, if given, lists the kept ranks in update order
    (method "full" only).  Returns (final MPS, records); each record also
    carries the key (b, tau) of the gate it applied.
    """
    state = mps0.copy()
    records = []
    n = state.n_sites
    sweep_id = 0
    for _ in range(steps):
        for parity, frac in om.STEP_SWEEPS:
            tau = frac * dt
            for b in range(parity, n - 1, 2):
                omega_of = None
                if method in ("rrsvd", "rrsvd_adaptive"):
                    ncol = state.dims[b + 1] * state.chis()[b + 2]

                    def omega_of(l, ncol=ncol, pid=chain * (n - 1) + b, sid=sweep_id):
                        return gaussian_omega(ncol, l, seed, pid, sid)
                fixed = None if schedule is None else schedule[len(records)]
                rec = recorded_bond_update(state, b, gate_fn(b, tau), chi_max, eps, method,
                                           omega_of, q, p, fixed, lambda_floor)
                rec["key"] = (b, tau)
                records.append(rec)
            sweep_id += 1
    return state, records


def expectation_with_seed(mps, op, site):
    """<O_site> by exact contraction and its cotangents w.r.t. every tensor.

    The contraction is ``mps.expectation`` restated with torch CPU float64 /
    complex128 ops so that autograd supplies dL/dGamma and dL/dlambda in the
    convention above (torch's complex gradient is dL/dx + i dL/dy).
    """
    import torch
    gs = [torch.tensor(np.array(g), dtype=torch.complex128, requires_grad=True) for g in mps.gammas]
    ls = [torch.tensor(np.array(l), dtype=torch.float64, requires_grad=True) for l in mps.lambdas]
    opt = torch.tensor(np.asarray(op, dtype=np.complex128))
    env_o = torch.ones((1, 1), dtype=torch.complex128)
    env_n = torch.ones((1, 1), dtype=torch.complex128)
    n = len(gs)
    for k in range(n):
        g = gs[k]
        a = g * ls[k].to(torch.complex128)[None, None, :] if k < n - 1 else g
        opk = opt if k == site else torch.eye(g.shape[0], dtype=torch.complex128)
        env_o = torch.einsum("ab,iac,ij,jbd->cd", env_o, a.conj(), opk, a)
        env_n = torch.einsum("ab,iac,ibd->cd", env_n, a.conj(), a)
    val = (env_o[0, 0] / env_n[0, 0]).real
    val.backward()
    return (float(val.item()), [g.grad.numpy().copy() for g in gs],
            [l.grad.numpy().copy() for l in ls])


def reverse_sweep(records, gammas_bar, lambdas_bar, n_sites, extra=None, lambda_floor=1e-14,
                  eta_rel=ETA_REL):
    """Run ``bond_adjoint`` over the records in reverse order.

    gammas_bar / lambdas_bar hold the cotangents of the final MPS and are
    updated in place to those of the initial one.  extra limits the
    discarded triplets coupled to the kept ones (None: all recorded).
    Returns {key: gate_bar} summed over every application of that gate.
    """
    gate_bars = {}
    for rec in reversed(records):
        b, chi = rec["b"], rec["chi"]
        r = len(rec["s"]) if extra is None else min(len(rec["s"]), chi + extra)
        out = bond_adjoint(rec["gk"], rec["gk1"], rec["lam_l"], rec["lam_m"], rec["lam_r"],
                           rec["gate"], rec["u"][:, :r], rec["s"][:r], rec["vh"][:r], chi,
                           gammas_bar[b], gammas_bar[b + 1], lambdas_bar[b], lambda_floor,
                           eta_rel)
        gammas_bar[b] = out["gk_bar"]
        gammas_bar[b + 1] = out["gk1_bar"]
        lambdas_bar[b] = out["lam_m_bar"]
        if b >= 1:
            lambdas_bar[b - 1] = lambdas_bar[b - 1] + out["lam_l_bar"]
        if b + 1 <= n_sites - 2:
            lambdas_bar[b + 1] = lambdas_bar[b + 1] + out["lam_r_bar"]
        key = rec["key"]
        gate_bars[key] = gate_bars.get(key, 0) + out["gate_bar"]
    return gate_bars


def expm_direction(x, e):
    """Frechet derivative of the matrix exponential at x in direction e.

    scipy's expm_frechet (block Pade of exp([[X, E], [0, X]])).
    """
    return scipy.linalg.expm_frechet(np.asarray(x, dtype=np.complex128),
                                     np.asarray(e, dtype=np.complex128), compute_expm=False)


def coupling_gradient(gate_bars, h_of, dh_of, n_params):
    """dL/dtheta_n = sum over gate keys (b, tau) of Re tr(Gbar^H dG/dtheta_n).

    G = exp(-i tau h_b(theta)); dG/dtheta_n is the Frechet derivative of exp
    at -i tau h_b in the direction -i tau dh_b/dtheta_n.  h_of(b) gives h_b,
    dh_of(b, n) its derivative (None when h_b does not depend on theta_n).
    """
    grad = np.zeros(n_params)
    for (b, tau), gbar in gate_bars.items():
        for n in range(n_params):
            dh = dh_of(b, n)
            if dh is None:
                continue
            dg = expm_direction(-1j * tau * h_of(b), -1j * tau * dh)
            grad[n] += float(np.real(np.sum(gbar.conj() * dg)))
    return grad


def tebd_gradient(mps0, gate_fn, h_of, dh_of, n_params, dt, steps, chi_max, eps, op, site,
                  method="full", q=2, p=10, seed=0, chain=0, extra=None, lambda_floor=1e-14,
                  eta_rel=ETA_REL):
    """<O_site(T)> and its gradient w.r.t. the couplings by reverse mode.

    Returns (value, gradient, records, final MPS).
    """
    final, records = run_recorded(mps0, gate_fn, dt, steps, chi_max, eps, method, q, p, seed,
                                  chain, lambda_floor=lambda_floor)
    val, gbar, lbar = expectation_with_seed(final, op, site)
    gate_bars = reverse_sweep(records, gbar, lbar, final.n_sites, extra, lambda_floor, eta_rel)
    return val, coupling_gradient(gate_bars, h_of, dh_of, n_params), records, final


def finite_difference_gradient(mps0, gate_fn_of, params, dt, steps, chi_max, eps, op, site,
                               schedule, h=1e-6, lambda_floor=1e-14):
    """Central differences of <O_site(T)> (O-def) with the kept ranks replayed.

    gate_fn_of(params) returns a gate function for those couplings.
    """
    params = np.asarray(params, dtype=np.float64)
    grad = np.zeros(len(params))
    for n in range(len(params)):
        vals = []
        for sign in (1.0, -1.0):
            pv = params.copy()
            pv[n] += sign * h
            final, _ = run_recorded(mps0, gate_fn_of(pv), dt, steps, chi_max, eps,
                                    schedule=schedule, lambda_floor=lambda_floor)
            vals.append(om.expectation(final, op, site).real)
        grad[n] = (vals[0] - vals[1]) / (2.0 * h)
    return grad
