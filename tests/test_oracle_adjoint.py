"""Pins of the oracle's reverse-mode derivative (``oracle.adjoint``).

The derivative is checked against central finite differences of the forward
maps (the definition of a derivative), and the gradient of a whole TEBD run
of the XX chain against the free-fermion closed form of the same Trotter
circuit, which carries no truncation.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import adjoint as oa
from oracle import freefermion as ff
from oracle import models as om
from oracle import mps as omps
from oracle import rrsvd as rr


def _cn(gen, *shape):
    return (gen.standard_normal(shape) + 1j * gen.standard_normal(shape)) / np.sqrt(2.0)


def _directional_fd(f, x, d, h=1e-6):
    return (f(x + h * d) - f(x - h * d)) / (2.0 * h)


def test_broadened_gaps():
    s = np.array([3.0, 2.0, 2.0, 0.5])
    f = oa.broadened_gaps(s, 1e-12 * 9.0)
    assert f[0, 1] == pytest.approx(1.0 / (4.0 - 9.0), rel=1e-15)
    assert f[3, 0] == pytest.approx(1.0 / (9.0 - 0.25), rel=1e-15)
    assert f[1, 2] == 0.0 and f[2, 1] == 0.0  # degenerate pair: finite (zero)
    assert np.all(np.diag(f) == 0.0)
    assert np.allclose(f, -f.T, atol=0)


def _svd_loss(gen, m, n, k):
    """A gauge-invariant loss of the kept triplets and its cotangents."""
    w1 = gen.standard_normal((m, k))
    w2 = gen.standard_normal((k, n))
    w3 = gen.standard_normal(k)
    w4 = _cn(gen, m, n)

    def loss(a):
        u, s, vh = rr.lapack_svd(a)
        u, s, vh = u[:, :k], s[:k], vh[:k]
        return (np.sum(w1 * np.abs(u) ** 2) + np.sum(w2 * np.abs(vh) ** 2) + w3 @ s
                + np.real(np.vdot(w4, u @ np.diag(s) @ vh)))

    def cotangents(u, s, vh):
        ubar = 2.0 * w1 * u + w4 @ vh.conj().T @ np.diag(s)
        vhbar = 2.0 * w2 * vh + np.diag(s) @ u.conj().T @ w4
        sbar = w3 + np.real(np.diag(u.conj().T @ w4 @ vh.conj().T))
        return ubar, sbar, vhbar
    return loss, cotangents


@pytest.mark.parametrize("m,n,rank,k", [(7, 5, 5, 5), (5, 8, 5, 5), (6, 6, 6, 6), (9, 7, 3, 3),
                                        (6, 10, 4, 4)])
def test_svd_backward_matches_finite_differences(m, n, rank, k):
    # k = rank: the kept triplets span A exactly, so the formula (with its
    # projector terms when k < min(m, n)) is the exact derivative.
    gen = np.random.default_rng(100 + m * n + k)
    a = _cn(gen, m, rank) @ _cn(gen, rank, n)
    loss, cot = _svd_loss(gen, m, n, k)
    u, s, vh = rr.lapack_svd(a)
    u, s, vh = u[:, :k], s[:k], vh[:k]
    abar = oa.svd_backward(u, s, vh, *cot(u, s, vh))
    for _ in range(4):
        d = _cn(gen, m, n)
        fd = _directional_fd(loss, a, d)
        assert abs(np.real(np.vdot(abar, d)) - fd) < 1e-7 * max(1.0, abs(fd))


def test_svd_backward_discarded_triplets_enter_with_zero_cotangent():
    # Truncating a full-rank matrix: coupling the kept triplets to all the
    # others gives the exact derivative of the truncated map; dropping them
    # (kept triplets only) does not.
    gen = np.random.default_rng(7)
    m, n, k = 8, 6, 3
    a = _cn(gen, m, n)
    loss, cot = _svd_loss(gen, m, n, k)
    u, s, vh = rr.lapack_svd(a)
    ubar, sbar, vhbar = cot(u[:, :k], s[:k], vh[:k])
    r = len(s)
    ub = np.zeros((m, r), complex)
    ub[:, :k] = ubar
    vb = np.zeros((r, n), complex)
    vb[:k] = vhbar
    sb = np.zeros(r)
    sb[:k] = sbar
    full = oa.svd_backward(u, s, vh, ub, sb, vb)
    kept = oa.svd_backward(u[:, :k], s[:k], vh[:k], ubar, sbar, vhbar)
    worst_full = worst_kept = 0.0
    for _ in range(4):
        d = _cn(gen, m, n)
        fd = _directional_fd(loss, a, d)
        worst_full = max(worst_full, abs(np.real(np.vdot(full, d)) - fd) / max(1.0, abs(fd)))
        worst_kept = max(worst_kept, abs(np.real(np.vdot(kept, d)) - fd) / max(1.0, abs(fd)))
    assert worst_full < 1e-7
    assert worst_kept > 1e-3


def _bond_case(gen, dl, dr, cl, cm, cr):
    gk, gk1, ll, lm, lr = wl.random_vidal_bond(dl, dr, cl, cm, cr, gen)
    gate = wl.random_unitary(dl * dr, gen)
    return [gk, gk1, ll, lm, lr, gate]


def _bond_forward(x, chi, floor=1e-14):
    """The bond update of ``mps.bond_update`` on explicit tensors, fixed chi'."""
    gk, gk1, ll, lm, lr, gate = x
    dl, cl, _ = gk.shape
    dr, _, cr = gk1.shape
    th = omps.apply_gate(gate, np.einsum("a,iag,g,jgc,c->ijac", ll, gk, lm, gk1, lr))
    u, s, vh = rr.lapack_svd(omps.blocked(th))
    inv_l, _ = omps.safe_inverse(ll, floor)
    inv_r, _ = omps.safe_inverse(lr, floor)
    gkn = u[:, :chi].reshape(dl, cl, chi) * inv_l[None, :, None]
    gk1n = vh[:chi].reshape(chi, dr, cr).transpose(1, 0, 2) * inv_r[None, None, :]
    lamn = s[:chi] / np.linalg.norm(s[:chi])
    return gkn, gk1n, lamn, (u, s, vh)


@pytest.mark.parametrize("shape,chi", [((2, 3, 3, 4, 2), None), ((2, 2, 3, 2, 3), None),
                                       ((3, 2, 2, 3, 4), 3)])
def test_bond_adjoint_matches_finite_differences(shape, chi):
    gen = np.random.default_rng(sum(shape))
    dl, dr, cl, cm, cr = shape
    x0 = _bond_case(gen, dl, dr, cl, cm, cr)
    full = min(dl * cl, dr * cr)
    chi = full if chi is None else chi
    # a gauge-invariant loss of the three outputs
    w1 = gen.standard_normal((dl, cl, chi))
    w2 = gen.standard_normal((dr, chi, cr))
    w3 = gen.standard_normal(chi)
    w4 = _cn(gen, dl, dr, cl, cr)

    def loss_and_cot(x):
        gkn, gk1n, lamn, fac = _bond_forward(x, chi)
        ll, lr = x[2], x[4]
        rec = np.einsum("a,iag,g,jgc,c->ijac", ll, gkn, lamn, gk1n, lr)
        val = (np.sum(w1 * np.abs(gkn) ** 2) + np.sum(w2 * np.abs(gk1n) ** 2) + w3 @ lamn
               + np.real(np.vdot(w4, rec)))
        gb = 2 * w1 * gkn + np.einsum("ijac,a,g,jgc,c->iag", w4, ll, lamn, gk1n.conj(), lr)
        g1b = 2 * w2 * gk1n + np.einsum("ijac,a,iag,g,c->jgc", w4, ll, gkn.conj(), lamn, lr)
        lb = w3 + np.einsum("ijac,a,iag,jgc,c->g", w4.conj(), ll, gkn, gk1n, lr).real
        # the reconstruction also reads lambda_l, lambda_r directly
        extra_l = np.einsum("ijac,iag,g,jgc,c->a", w4.conj(), gkn, lamn, gk1n, lr).real
        extra_r = np.einsum("ijac,a,iag,g,jgc->c", w4.conj(), ll, gkn, lamn, gk1n).real
        return val, fac, gb, g1b, lb, extra_l, extra_r

    _, (u, s, vh), gb, g1b, lb, extra_l, extra_r = loss_and_cot(x0)
    out = oa.bond_adjoint(*x0, u, s, vh, chi, gb, g1b, lb)
    bars = [out["gk_bar"], out["gk1_bar"], out["lam_l_bar"] + extra_l, out["lam_m_bar"],
            out["lam_r_bar"] + extra_r, out["gate_bar"]]
    for idx in range(6):
        for _ in range(2):
            cplx = np.iscomplexobj(x0[idx])
            d = _cn(gen, *x0[idx].shape) if cplx else gen.standard_normal(x0[idx].shape)

            def f(v):
                x = list(x0)
                x[idx] = v
                return loss_and_cot(x)[0]
            fd = _directional_fd(f, x0[idx], d)
            an = np.real(np.vdot(bars[idx], d)) if cplx else float(bars[idx] @ d)
            assert abs(an - fd) < 1e-7 * max(1.0, abs(fd)), (idx, an, fd)


def test_bond_adjoint_lambda_floor_rows_carry_no_cotangent():
    gen = np.random.default_rng(11)
    x = _bond_case(gen, 2, 2, 3, 3, 3)
    x[2] = np.array([0.9, 0.43, 1e-16])  # lambda_l below the floor in one entry
    gkn, gk1n, lamn, (u, s, vh) = _bond_forward(x, 4)
    assert np.all(gkn[:, 2, :] == 0)
    gb = _cn(gen, *gkn.shape)
    out = oa.bond_adjoint(*x, u, s, vh, 4, gb, np.zeros_like(gk1n), np.zeros(4))
    out2 = oa.bond_adjoint(*x, u, s, vh, 4, gb * np.array([1, 1, 0])[None, :, None],
                           np.zeros_like(gk1n), np.zeros(4))
    # the cotangent of a Gamma' row that was zeroed by the floor is ignored
    for key in ("gk_bar", "gk1_bar", "lam_m_bar", "gate_bar"):
        assert np.allclose(out[key], out2[key], atol=1e-13)


def test_expectation_seed_matches_finite_differences():
    gen = np.random.default_rng(5)
    dims, chis = [2, 3, 2, 2], [1, 2, 3, 2, 1]
    gam = [_cn(gen, dims[k], chis[k], chis[k + 1]) for k in range(4)]
    lam = [np.sort(gen.uniform(0.2, 1.0, chis[k + 1]))[::-1] for k in range(3)]
    op = np.diag([1.0, -1.0, 0.5])[:3, :3]
    state = omps.MPS(gam, lam)
    val, gbar, lbar = oa.expectation_with_seed(state, op, 1)
    assert val == pytest.approx(omps.expectation(state, op, 1).real, abs=1e-14)
    for k in range(4):
        d = _cn(gen, *gam[k].shape)

        def f(v, k=k):
            g2 = list(gam)
            g2[k] = v
            return omps.expectation(omps.MPS(g2, lam), op, 1).real
        fd = _directional_fd(f, gam[k], d)
        assert abs(np.real(np.vdot(gbar[k], d)) - fd) < 1e-8
    for k in range(3):
        d = gen.standard_normal(lam[k].shape)

        def f(v, k=k):
            l2 = list(lam)
            l2[k] = v
            return omps.expectation(omps.MPS(gam, l2), op, 1).real
        assert abs(float(lbar[k] @ d) - _directional_fd(f, lam[k], d)) < 1e-8


def test_expm_direction_matches_finite_differences():
    gen = np.random.default_rng(9)
    h = _cn(gen, 4, 4)
    h = h + h.conj().T
    e = _cn(gen, 4, 4)
    e = e + e.conj().T
    tau = 0.3
    got = oa.expm_direction(-1j * tau * h, -1j * tau * e)
    fd = (om.gate(h + 1e-6 * e, tau) - om.gate(h - 1e-6 * e, tau)) / 2e-6
    assert np.max(np.abs(got - fd)) < 1e-9


# ---------------------------------------------------------------------------
# Whole TEBD runs of the XX chain with random fields (gradient of <Z_0(T)>
# with respect to the bond couplings J_b).

HOP = 0.5 * (np.kron(om.X, om.X) + np.kron(om.Y, om.Y))


def _xx_problem(n_sites, seed=wl.BASE_SEED):
    couplings, fields = wl.xx_couplings(n_sites, seed=seed)

    def gate_fn_of(jv):
        hb = om.xx_field(jv, fields)[1]
        cache = {}

        def g(b, tau):
            if (b, tau) not in cache:
                cache[(b, tau)] = om.gate(hb[b], tau)
            return cache[(b, tau)]
        return g
    dims, hb = om.xx_field(couplings, fields)
    mps0 = omps.basis_product_state(dims, wl.neel_levels(n_sites))
    return couplings, fields, gate_fn_of, hb, mps0


def test_free_fermion_gradient_reference_converged():
    J, h = wl.xx_couplings(6, seed=3)
    g1 = ff.z_gradient(J, h, wl.neel_levels(6), 0.02, 10, h=1e-3)
    g2 = ff.z_gradient(J, h, wl.neel_levels(6), 0.02, 10, h=5e-4)
    assert np.max(np.abs(g1 - g2)) < 1e-11
    # a coupling far outside the light cone of site 0 has a tiny derivative
    assert abs(g1[-1]) < 1e-6 * np.max(np.abs(g1))


@pytest.mark.parametrize("n_sites,steps", [(8, 15)])
def test_tebd_gradient_matches_fd_and_free_fermion(n_sites, steps):
    dt, chi_max, eps = 0.02, 32, 1e-10
    J, h, gate_fn_of, hb, mps0 = _xx_problem(n_sites)
    val, grad, recs, _ = oa.tebd_gradient(mps0, gate_fn_of(J), lambda b: hb[b],
                                          lambda b, n: HOP if b == n else None, n_sites - 1,
                                          dt, steps, chi_max, eps, om.Z, 0)
    assert max(r["chi"] for r in recs) < chi_max  # truncation by the tolerance only
    sched = [r["chi"] for r in recs]
    fd = oa.finite_difference_gradient(mps0, gate_fn_of, J, dt, steps, chi_max, eps, om.Z, 0,
                                       sched)
    scale = np.max(np.abs(fd))
    assert np.max(np.abs(grad - fd)) < 1e-7 * scale
    ffg = ff.z_gradient(J, h, wl.neel_levels(n_sites), dt, steps)
    assert val == pytest.approx(ff.z_profile(J, h, wl.neel_levels(n_sites), dt, steps)[0],
                                abs=1e-7)
    assert np.max(np.abs(grad - ffg)) < 1e-5 * scale
    # coupling only to the kept triplets is a coarser approximation
    _, gb, lb = oa.expectation_with_seed(oa.run_recorded(mps0, gate_fn_of(J), dt, steps,
                                                         chi_max, eps)[0], om.Z, 0)
    kept = oa.coupling_gradient(oa.reverse_sweep(recs, gb, lb, n_sites, extra=0),
                                lambda b: hb[b], lambda b, n: HOP if b == n else None,
                                n_sites - 1)
    assert np.max(np.abs(kept - fd)) > np.max(np.abs(grad - fd))


def test_tebd_gradient_rrsvd_adaptive_matches_exact_svd():
    n_sites, steps, dt = 8, 10, 0.02
    J, h, gate_fn_of, hb, mps0 = _xx_problem(n_sites, seed=21)
    args = (mps0, gate_fn_of(J), lambda b: hb[b], lambda b, n: HOP if b == n else None,
            n_sites - 1, dt, steps, 32, 1e-10, om.Z, 0)
    v_full, g_full, _, _ = oa.tebd_gradient(*args)
    v_rr, g_rr, recs, _ = oa.tebd_gradient(*args, method="rrsvd_adaptive", seed=77)
    assert abs(v_rr - v_full) < 1e-12
    assert np.max(np.abs(g_rr - g_full)) < 1e-9 * np.max(np.abs(g_full))
    assert all(len(r["s"]) >= r["chi"] for r in recs)
