"""Pins of the Accuracy Check oracle (Sec. IV: Theorem 2, Alg. 2, Fact 1).

* Theorem 2's constant: for a rank-one M = u v^H, ||M w|| = |v^H w| with
  v^H w ~ CN(0, 1), so P(||M|| > c max_i ||M w_i||) = (1 - exp(-1/c^2))^r
  exactly; the oracle's constant must reproduce that frequency (a wrong
  constant or a dropped square root fails), and the bound must hold with
  probability >= 1 - 10^-r on a full-rank M.
* Fact 1: sigma_j = sigma_1 / j gives sum 1/j^2 -> pi^2/6 (Basel).
* Alg. 2: from a too-small basis the check grows Q until the true Frobenius
  residual meets the target; it stops at l > n - r; it does nothing when
  the basis is already good.
* The RRSVD with the check equals the exact truncated SVD of TEBD-like
  matrices, and the TEBD method built on it reproduces full-SVD TEBD.
"""
import numpy as np

import workloads as wl
from oracle import models, mps, philox, rrsvd as rr


def _gauss(n, r, gen):
    return (gen.standard_normal((n, r)) + 1j * gen.standard_normal((n, r))) / np.sqrt(2.0)


def test_theorem2_constant_rank_one_frequency():
    gen = np.random.default_rng(5)
    n, trials, r = 40, 200000, 1
    v = np.ones(n) / np.sqrt(n)
    w = _gauss(n, trials, gen)
    proj = np.abs(v @ w)  # ||M w|| for M = u v^H, ||M|| = 1
    fail = np.mean(rr.THEOREM2_CONST * proj < 1.0)
    expect = 1.0 - np.exp(-1.0 / rr.THEOREM2_CONST ** 2)
    assert abs(fail - expect) < 5 * np.sqrt(expect / trials)
    assert expect < 10.0 ** -r


def test_theorem2_bound_holds_on_full_rank_residuals():
    gen = np.random.default_rng(6)
    fails = 0
    for t in range(300):
        a = wl.known_spectrum(60, 50, np.exp(-np.arange(50) / 8.0), gen)
        q, _ = np.linalg.qr(a @ _gauss(50, 6, gen))
        m = a - q @ (q.conj().T @ a)
        est, _ = rr.probe_residual(a, q, _gauss(50, 2, gen))
        fails += np.linalg.norm(m, 2) > rr.THEOREM2_CONST * est
    assert fails <= 3  # probability <= 1e-2 per trial


def test_fact1_basel_bound():
    for n in (10, 1000, 100000):
        s = 1.0 / np.arange(1, n + 1)
        f = np.sqrt(np.sum(s ** 2))
        assert f <= rr.FACT1_CONST + 1e-15
    assert abs(np.sqrt(np.sum(1.0 / np.arange(1, 10 ** 6 + 1) ** 2)) - rr.FACT1_CONST) < 1e-6
    gen = np.random.default_rng(7)
    s = np.sort(gen.uniform(0, 1, 300) / np.arange(1, 301))[::-1]
    s = np.minimum(s, s[0] / np.arange(1, 301))
    assert np.sqrt(np.sum(s ** 2)) <= rr.FACT1_CONST * s[0]
    assert rr.ACC_CONST >= rr.THEOREM2_CONST * rr.FACT1_CONST


def _probe_of(n, seed=1504, pid=3):
    return lambda c0, w: philox.gaussian_omega(n, c0 + w, seed, pid, 0)[:, c0:]


def test_accuracy_check_grows_basis_to_target():
    gen = wl.rng(11)
    n = 200
    a = wl.known_spectrum(n, n, np.exp(-np.arange(n) / 5.0), gen)
    frob = np.linalg.norm(a)
    eps = 1e-10
    q0 = rr.range_basis(a @ _probe_of(n)(0, 15))
    tol = np.sqrt(eps) * frob / rr.ACC_CONST
    q, rounds, capped, hist = rr.accuracy_check(a, q0, 10, tol, _probe_of(n), n, 15)
    assert rounds > 0 and not capped and hist[-1] <= tol
    resid = np.linalg.norm(a - q @ (q.conj().T @ a))
    assert resid <= np.sqrt(eps) * frob
    # needed ~ 5 ln(1e5 * ...) columns; the check stops within two blocks of it
    need = int(np.sum(np.exp(-np.arange(n) / 5.0) > 1e-5 * np.exp(0) / rr.ACC_CONST))
    assert q.shape[1] <= need + 20
    assert np.allclose(q.conj().T @ q, np.eye(q.shape[1]), atol=1e-12)
    # a basis that already meets the target is returned as it is
    q2, rounds2, _, _ = rr.accuracy_check(a, q, 10, tol, _probe_of(n), n, 200)
    assert rounds2 == 0 and q2.shape == q.shape


def test_accuracy_check_stops_at_n_minus_r():
    gen = wl.rng(12)
    n = 30
    a = wl.known_spectrum(n, n, np.linspace(1.0, 0.5, n), gen)  # flat: never meets 1e-10
    q0 = rr.range_basis(a @ _probe_of(n)(0, 5))
    q, rounds, capped, hist = rr.accuracy_check(a, q0, 10, 1e-6, _probe_of(n), n, 5)
    assert q.shape[1] == 25 and rounds == 2 and not capped  # 5 -> 15 -> 25 > n - r
    # a capacity of 12: the first block is cut to 7 columns, then the check stops
    q, rounds, capped, _ = rr.accuracy_check(a, q0, 10, 1e-6, _probe_of(n), 12, 5)
    assert capped and rounds == 1 and q.shape[1] == 12


def test_rrsvd_accuracy_equals_exact_truncation():
    gen = wl.rng(13)
    for (m, n, decay) in ((120, 90, 4.0), (60, 200, 7.0)):
        a = wl.known_spectrum(m, n, np.exp(-np.arange(min(m, n)) / decay), gen)
        u, s, vh, chi, w, st, rounds = rr.truncate_rrsvd_accuracy(a, _probe_of(n), 2, 64, 1e-10, 3, 10, 10)
        _, sd, _, cd, wd, _ = rr.truncate_full_svd(a, 64, 1e-10)
        assert rounds > 0 and chi == cd and abs(w - wd) < 1e-12
        assert np.max(np.abs(s - sd)) < 1e-10 * sd[0]


def test_accuracy_tebd_matches_full_svd_tebd():
    n, dt, steps = 8, 0.05, 10
    dims, hb = models.tfim(n, 1.0, 1.0)
    gates = {}

    def gfn(b, tau):
        if (b, tau) not in gates:
            gates[(b, tau)] = models.gate(hb[b], tau)
        return gates[(b, tau)]
    runs = {}
    for method in ("full", "rrsvd_accuracy"):
        drv = mps.TEBD(mps.basis_product_state(dims, [0] * n), gfn, dt, 16, 1e-10, method=method,
                       p=4, q=2, seed=1504)
        for _ in range(steps):
            drv.step()
        runs[method] = drv.mps
    assert runs["full"].chis() == runs["rrsvd_accuracy"].chis()
    for i in range(n):
        za = mps.expectation(runs["full"], models.Z, i).real
        zb = mps.expectation(runs["rrsvd_accuracy"], models.Z, i).real
        assert abs(za - zb) < 1e-10
