"""Pins of the oracle's truncated SVD (O-def) and step-by-step RRSVD (O-alg)."""
import numpy as np
import pytest

import workloads as wl
from oracle import philox, rrsvd


def _known(m, n, s, seed):
    return wl.known_spectrum(m, n, s, wl.rng(seed))


def test_full_svd_recovers_known_spectrum_and_eckart_young():
    s = np.exp(-np.arange(60) / 6.0)
    a = _known(90, 60, s, 1)
    u, sk, vh, chi, w, st = rrsvd.truncate_full_svd(a, chi_max=100, eps=1e-8)
    assert np.allclose(sk, s[:chi], atol=1e-14, rtol=0)
    # Eckart-Young: the residual of the rank-chi' factors is the discarded tail
    resid = a - (u * sk[None, :]) @ vh
    assert np.linalg.norm(resid) ** 2 == pytest.approx(np.sum(s[chi:] ** 2), rel=1e-9, abs=1e-28)
    assert w == pytest.approx(np.sum(s[chi:] ** 2) / np.sum(s ** 2), rel=1e-9)
    assert w <= 1e-8 < np.sum(s[chi - 1:] ** 2) / np.sum(s ** 2)
    # orthonormal factors
    assert np.allclose(u.conj().T @ u, np.eye(chi), atol=1e-13)
    assert np.allclose(vh @ vh.conj().T, np.eye(chi), atol=1e-13)


def test_rrsvd_exact_when_sketch_spans_range():
    # l = min(k + p, m, n) = n: span(Y) is the whole range, RRSVD is exact.
    s = np.exp(-np.arange(30) / 4.0)
    a = _known(50, 30, s, 2)
    l = rrsvd.sketch_width(32, 10, 50, 30)
    assert l == 30
    om = philox.gaussian_omega(30, l, 7, 0, 0)
    u, sv, vh = rrsvd.rrsvd(a, om, q=2)
    assert np.allclose(sv, s, atol=1e-14, rtol=0)
    assert np.allclose((u * sv[None, :]) @ vh, a, atol=1e-13)


def test_rrsvd_rank_deficient_input():
    # Rank 5 < l: Y is exactly rank deficient; the range finder keeps the 5
    # informative directions and the 5 nonzero singular values are exact.
    s = np.array([1.0, 0.7, 0.3, 0.1, 0.01])
    a = _known(40, 40, s, 3)
    om = philox.gaussian_omega(40, 15, 9, 1, 0)
    q = rrsvd.rrsvd_range(a, om, 2)
    assert q.shape == (40, 5)
    assert np.allclose(q.conj().T @ q, np.eye(5), atol=1e-13)
    u, sv, vh = rrsvd.rrsvd(a, om, 2)
    assert len(sv) == 5 and np.allclose(sv, s, atol=1e-14)
    assert np.allclose((u * sv[None, :]) @ vh, a, atol=1e-13)


def test_power_iteration_subspace_matches_unorthogonalised_product():
    # Eq. (Z): span(Q_q) = span((A A^H)^q A Omega).  On a well-conditioned A
    # the product can be formed directly; the projectors must agree.
    s = np.linspace(1.0, 0.5, 20)
    a = _known(30, 20, s, 4)
    om = philox.gaussian_omega(20, 6, 11, 0, 0)
    for q in (0, 1, 2):
        z = a @ om
        for _ in range(q):
            z = a @ (a.conj().T @ z)
        qz, _ = np.linalg.qr(z)
        qq = rrsvd.rrsvd_range(a, om, q)
        assert np.allclose(qq @ qq.conj().T, qz @ qz.conj().T, atol=1e-11)
    # and a different q gives a different subspace
    q1 = rrsvd.rrsvd_range(a, om, 1)
    q2 = rrsvd.rrsvd_range(a, om, 2)
    assert not np.allclose(q1 @ q1.conj().T, q2 @ q2.conj().T, atol=1e-6)


def test_power_iteration_singular_values_raised():
    # Eq. (powSV): sigma_j((A A^H)^q A) = sigma_j(A)^(2q+1).
    s = np.linspace(1.0, 0.6, 12)
    a = _known(20, 12, s, 5)
    b = a.copy()
    for _ in range(2):
        b = a @ (a.conj().T @ b)
    sb = rrsvd.lapack_svd(b)[1]
    assert np.allclose(sb, s ** 5, atol=1e-13)


def test_rrsvd_ritz_values_interlace_and_meet_theorem_bound():
    # The RRSVD values are Ritz values: sigma_hat_j <= sigma_j.  Their quality
    # obeys Theorem 1 (expected range error), here checked with a x10 margin.
    n, k, p, q = 256, 64, 10, 2
    s = wl.exp_spectrum(n)
    a = _known(n, n, s, 6)
    om = philox.gaussian_omega(n, k + p, 1504, 0, 0)
    qm = rrsvd.rrsvd_range(a, om, q)
    u, sv, vh = rrsvd.rrsvd(a, om, q)
    assert np.all(sv <= s[:k + p] + 1e-14)
    err = np.linalg.norm(a - qm @ (qm.conj().T @ a), 2)
    tail = s[k:]
    bound = ((1 + np.sqrt(k / (p - 1))) * s[k] ** (2 * q + 1)
             + np.e * np.sqrt(k + p) / p * np.sqrt(np.sum(tail ** (2 * (2 * q + 1))))) ** (1 / (2 * q + 1))
    assert err <= 10 * bound
    assert err >= s[k + p] * 0.999  # no rank-l subspace beats sigma_{l+1}
    # leading values are accurate to rounding
    assert np.max(np.abs(sv[:20] - s[:20])) < 1e-10


def test_truncate_rrsvd_weight_uses_frobenius_identity():
    s = np.exp(-np.arange(80) / 5.0)
    a = _known(100, 80, s, 7)
    om = philox.gaussian_omega(80, 40, 3, 2, 1)
    u, sk, vh, chi, w, st = rrsvd.truncate_rrsvd(a, om, 2, chi_max=30, eps=1e-10)
    resid = a - (u * sk[None, :]) @ vh
    assert w * np.sum(s ** 2) == pytest.approx(np.linalg.norm(resid) ** 2, rel=1e-6, abs=1e-24)
    chi_def = rrsvd.truncate_full_svd(a, 30, 1e-10)[3]
    assert chi == chi_def


def test_range_basis_keeps_the_numerical_rank():
    gen = wl.rng(12)
    # exact rank 7 sketch of 40 columns: 7 directions kept, and they span Y
    y = wl.ginibre(60, 7, gen) @ wl.ginibre(7, 40, gen)
    q = rrsvd.range_basis(y)
    assert q.shape == (60, 7)
    assert np.allclose(q.conj().T @ q, np.eye(7), atol=1e-13)
    assert np.allclose(q @ (q.conj().T @ y), y, atol=1e-12 * np.linalg.norm(y))
    # full-rank, well-conditioned: same subspace as the unpivoted QR
    y = wl.ginibre(50, 12, gen)
    q = rrsvd.range_basis(y)
    q0, _ = np.linalg.qr(y)
    assert q.shape == (50, 12) and np.allclose(q @ q.conj().T, q0 @ q0.conj().T, atol=1e-12)
    # graded columns below the tolerance are dropped, above it kept
    u = haar = wl.haar_isometry(30, 6, gen)
    sv = np.array([1.0, 1e-3, 1e-8, 1e-12, 1e-15, 1e-17])
    y = (u * sv[None, :]) @ wl.haar_isometry(6, 6, gen).conj().T
    assert rrsvd.range_basis(y).shape[1] == 4
    # the zero matrix keeps one (arbitrary) direction
    assert rrsvd.range_basis(np.zeros((5, 3), dtype=np.complex128)).shape[1] == 1


def test_adaptive_two_stage_rule():
    # A spectrum whose tolerance is met at rank 9: a first stage with k1 = 12
    # suffices; with k1 = 6 the rule must fall back to the fixed-rank width and
    # reproduce the fixed-rank result exactly (same test-matrix columns).
    s = np.exp(-np.arange(80) / 0.8)
    a = _known(90, 80, s, 13)
    omega_of = lambda l: philox.gaussian_omega(80, l, 5, 1, 2)
    eps = 1e-10
    chi_def = rrsvd.truncate_full_svd(a, 40, eps)[3]
    u, sv, vh, chi, w, st, stage = rrsvd.truncate_rrsvd_adaptive(a, omega_of, 2, 40, eps, 12, 10)
    assert stage == 1 and chi == chi_def <= 12 and w <= eps
    # the Frobenius identity carries an absolute rounding error of ~1e-14
    assert np.linalg.norm(a - (u * sv[None, :]) @ vh) ** 2 / np.sum(s ** 2) == pytest.approx(w, abs=1e-13)
    u2, sv2, vh2, chi2, w2, st2, stage2 = rrsvd.truncate_rrsvd_adaptive(a, omega_of, 2, 40, eps, 6, 10)
    assert stage2 == 2
    fixed = rrsvd.truncate_rrsvd(a, omega_of(50), 2, 40, eps)
    assert chi2 == fixed[3] and np.array_equal(sv2, fixed[1]) and w2 == fixed[4]
    # first-stage rank: chi + max(4, ceil(chi/4)), capped
    assert rrsvd.first_stage_rank(1, 100) == 5 and rrsvd.first_stage_rank(19, 100) == 24
    assert rrsvd.first_stage_rank(40, 100) == 50
    assert rrsvd.first_stage_rank(90, 100) == 100
