"""Pins of the oracle's generator and truncation rule (CPU only)."""
import os

import numpy as np
import pytest

from oracle import philox, rrsvd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_kv(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32_10(np.array(r[0:4], dtype=np.uint64), (r[4], r[5]))
        assert [int(x) for x in out] == r[6:10]


def test_gaussian_omega_statistics_and_streams():
    om = philox.gaussian_omega(400, 50, seed=1504, problem=3, call=7)
    assert om.shape == (400, 50) and om.dtype == np.complex128
    # complex standard normal: E z = 0, E|z|^2 = 1, Re and Im each variance 1/2
    assert abs(om.mean()) < 0.02
    assert abs(np.mean(np.abs(om) ** 2) - 1.0) < 0.02
    assert abs(np.var(om.real) - 0.5) < 0.02 and abs(np.var(om.imag) - 0.5) < 0.02
    assert abs(np.mean(om.real * om.imag)) < 0.02
    # deterministic and element-addressed: a sub-block equals a smaller draw
    again = philox.gaussian_omega(100, 20, seed=1504, problem=3, call=7)
    assert np.array_equal(om[:100, :20], again)
    # other problem / call / seed give unrelated draws
    for kw in ({"problem": 4, "call": 7, "seed": 1504}, {"problem": 3, "call": 8, "seed": 1504},
               {"problem": 3, "call": 7, "seed": 1505}):
        other = philox.gaussian_omega(100, 20, **kw)
        assert abs(np.vdot(other, again)) / 2000 < 0.1


def test_uniform_open_interval():
    u = philox.uniform_open01(np.array([0, 0xFFFFFFFF], dtype=np.uint64))
    assert 0.0 < u[0] < 1e-9 and 1.0 - 1e-9 < u[1] < 1.0


def test_critical_spectrum_printed_values():
    g = _read_kv("critical_spectrum.txt")
    n, k = int(g["n"]), int(g["k"])
    s = 1.0 / np.arange(1, n + 1)
    frob2 = np.sum(s ** 2)
    chi, w, status = rrsvd.truncation_rank(rrsvd.tail_weights(s), chi_max=k, eps=1e-300)
    assert chi == k and status == rrsvd.STATUS_CHI_BOUND
    err = np.sqrt(w)
    assert 0.5 * g["error_at_k_approx"] < err < 2.0 * g["error_at_k_approx"]
    chi2, w2, status2 = rrsvd.truncation_rank(rrsvd.tail_weights(s), chi_max=n, eps=g["target_error"] ** 2)
    assert status2 == 0 and np.sqrt(w2) <= g["target_error"]
    assert abs(chi2 - g["kept_for_target_approx"]) <= 0.05 * g["kept_for_target_approx"]
    # the rank just below chi2 misses the target (smallest c)
    assert np.sqrt(np.sum(s[chi2 - 1:] ** 2) / frob2) > g["target_error"]


def test_fact1_frobenius_bound():
    # Fact 1 (Sec. IV): sigma_j <= sigma_1 / j  =>  ||A||_F <= pi/sqrt(6) sigma_1.
    s = 1.0 / np.arange(1, 751)
    assert np.sqrt(np.sum(s ** 2)) <= np.pi / np.sqrt(6.0)
    assert np.sqrt(np.sum(s ** 2)) > 0.99 * np.pi / np.sqrt(6.0)


@pytest.mark.parametrize("eps", [1e-10, 1e-4, 0.3])
def test_truncation_rank_is_smallest_rank_meeting_target(eps):
    s = np.exp(-0.5 * np.arange(40))
    frob2 = np.sum(s ** 2)
    chi, w, st = rrsvd.truncation_rank(rrsvd.tail_weights(s), chi_max=100, eps=eps)
    chi_f, w_f, st_f = rrsvd.truncation_rank(rrsvd.frobenius_weights(s, frob2), chi_max=100, eps=eps)
    assert (chi_f, st_f) == (chi, st) and abs(w_f - w) < 1e-15
    brute = [c for c in range(1, 41) if np.sum(s[c:] ** 2) / frob2 <= eps][0]
    assert chi == brute and st == 0
    assert w == pytest.approx(np.sum(s[chi:] ** 2) / frob2, abs=1e-15)


def test_truncation_rank_edge_cases():
    tw = rrsvd.tail_weights
    # all weight in the first value: chi' = 1, w = 0
    chi, w, st = rrsvd.truncation_rank(tw(np.array([2.0, 0.0, 0.0])), 10, 1e-10)
    assert (chi, st) == (1, 0) and w == 0.0
    # chi_max binds
    chi, w, st = rrsvd.truncation_rank(tw(np.ones(8)), 3, 1e-10)
    assert chi == 3 and st == rrsvd.STATUS_CHI_BOUND and w == pytest.approx(5 / 8)
    # fewer values than chi_max and the target unreachable within them
    chi, w, st = rrsvd.truncation_rank(rrsvd.frobenius_weights(np.ones(4), 8.0), 10, 1e-10)
    assert chi == 4 and st == rrsvd.STATUS_CHI_BOUND and w == pytest.approx(0.5)
    # fixed rank (eps <= 0)
    chi, w, st = rrsvd.truncation_rank(tw(np.ones(4)), 3, 0.0)
    assert chi == 3 and st == 0 and w == pytest.approx(0.25)
    # zero matrix
    chi, w, st = rrsvd.truncation_rank(rrsvd.frobenius_weights(np.zeros(4), 0.0), 3, 1e-10)
    assert chi == 1 and w == 0.0
    # ties at the cut: the rule counts values, the result is still the smallest c
    s = np.array([1.0, 0.5, 0.5, 1e-9])
    chi, w, st = rrsvd.truncation_rank(tw(s), 10, 1e-12)
    assert chi == 3


def test_tail_weights_resolve_below_rounding_of_the_identity():
    # The plain tail sum resolves weights far below 1e-16; the Frobenius
    # identity cannot (cancellation), which is why O-def uses the tail sum.
    s = np.array([1.0, 1e-9, 1e-12])
    w = rrsvd.tail_weights(s)
    assert w[0] == pytest.approx(1e-18 + 1e-24, rel=1e-12)
    assert w[1] == pytest.approx(1e-24, rel=1e-12)
