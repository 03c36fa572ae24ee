"""Pins of the oracle's MPS bond update and TEBD driver (CPU only)."""
import numpy as np
import pytest

import workloads as wl
from oracle import freefermion, models, mps, philox, rrsvd, statevector


def _random_mps(dims, chis, seed):
    gen = wl.rng(seed)
    gammas = []
    for k, d in enumerate(dims):
        gammas.append(wl.ginibre(d * chis[k], chis[k + 1], gen).reshape(d, chis[k], chis[k + 1]))
    lambdas = []
    for b in range(len(dims) - 1):
        v = np.sort(gen.uniform(0.2, 1.0, size=chis[b + 1]))[::-1]
        lambdas.append(v / np.linalg.norm(v))
    return mps.MPS(gammas, lambdas)


@pytest.mark.parametrize("method", ["full", "rrsvd"])
def test_bond_update_equals_gate_on_state_vector(method):
    # No truncation: the updated MPS must be G applied to the state vector
    # (up to the renormalisation 1/||Theta~||_F), for mixed local dims.
    dims = [2, 3, 3, 2, 3]
    chis = [1, 2, 4, 5, 3, 1]
    m0 = _random_mps(dims, chis, 10)
    psi0 = mps.to_statevector(m0)
    gen = wl.rng(11)
    for b in range(len(dims) - 1):
        g = wl.random_unitary(dims[b] * dims[b + 1], gen)
        m1 = m0.copy()
        om = None
        if method == "rrsvd":
            mm = dims[b] * chis[b]
            nn = dims[b + 1] * chis[b + 2]
            om = philox.gaussian_omega(nn, min(mm, nn), 5, b, 0)
        info = mps.bond_update(m1, b, g, chi_max=100, eps=0.0, method=method, omega=om)
        psi1 = mps.to_statevector(m1)
        want = statevector.apply_two_site(psi0, g, b, dims)
        assert np.allclose(psi1 * np.sqrt(info["frob2"]), want, atol=1e-12)
        assert info["w"] < 1e-14  # rounding of ||A||_F^2 - sum s^2 in the rrsvd branch


def test_theta_matches_brute_force_contraction():
    dims = [2, 3, 2]
    chis = [1, 2, 3, 1]
    m0 = _random_mps(dims, chis, 12)
    th = mps.theta(m0, 0)  # (d0, d1, 1, chi_r)
    psi = mps.to_statevector(m0).reshape(2, 3, 2)
    # contract the remaining site by hand: psi[i,j,k] = sum_c Theta(i,j,0,c)/lam_r[c] * lam_r...
    lam_r = m0.lambdas[1]
    g2 = m0.gammas[2][:, :, 0]  # (d2, chi_2)
    want = np.einsum("ijc,c,kc->ijk", th[:, :, 0, :] / lam_r[None, None, :], lam_r, g2)
    assert np.allclose(psi, want, atol=1e-13)
    a = mps.blocked(mps.apply_gate(np.eye(6), th))
    assert a.shape == (2 * 1, 3 * 3)
    assert np.allclose(a.reshape(2, 1, 3, 3).transpose(0, 2, 1, 3), th)


def _tfim_driver(n, dt, chi_max, eps, method, seed=0):
    dims, hb = models.tfim(n, 1.0, 1.0)
    m = mps.basis_product_state(dims, [0] * n)
    gates = {}

    def gfn(b, tau):
        key = (b, tau)
        if key not in gates:
            gates[key] = models.gate(hb[b], tau)
        return gates[key]
    return dims, hb, mps.TEBD(m, gfn, dt, chi_max, eps, method=method, p=10, q=2, seed=seed)


@pytest.mark.parametrize("method", ["full", "rrsvd"])
def test_tebd_equals_trotter_state_vector(method):
    n, dt, steps = 8, 0.05, 12
    dims, hb, drv = _tfim_driver(n, dt, 32, 0.0, method)  # eps <= 0: keep every value (chi <= 16 here)
    for _ in range(steps):
        drv.step()
    psi_mps = mps.to_statevector(drv.mps)
    psi_sv = statevector.trotter_evolve(statevector.product_vector(dims, [0] * n), hb, dims, dt, steps)
    ov = abs(np.vdot(psi_sv, psi_mps)) / (np.linalg.norm(psi_sv) * np.linalg.norm(psi_mps))
    assert abs(1 - ov) < 1e-12
    for site in (0, 3, 7):
        e_mps = mps.expectation(drv.mps, models.Z, site).real
        e_sv = statevector.local_expectation(psi_sv, models.Z, site, dims).real
        assert abs(e_mps - e_sv) < 1e-11
    # canonical form is kept: norm 1 and the local formula agrees
    assert abs(mps.norm2(drv.mps) - 1) < 1e-12
    assert abs(mps.local_expectation_canonical(drv.mps, models.Z, 3).real
               - mps.expectation(drv.mps, models.Z, 3).real) < 1e-11
    # lambdas are the Schmidt values of the state at each cut
    for b in (1, 3, 5):
        sch = statevector.schmidt_values(psi_sv / np.linalg.norm(psi_sv), b, dims)
        lam = drv.mps.lambdas[b]
        assert np.allclose(lam, sch[:len(lam)], atol=1e-11)
        assert np.sum(sch[len(lam):] ** 2) < 1e-14


def test_trotter_error_is_second_order():
    # Eq. (defst3rd) splitting: global error O(dt^2); halving dt divides it by ~4.
    n, T = 6, 0.8
    dims, hb = models.tfim(n, 1.0, 1.0)
    H = models.full_hamiltonian(dims, hb)
    psi0 = statevector.product_vector(dims, [0] * n)
    exact = statevector.exact_evolve(psi0, H, T)
    errs = []
    for steps in (8, 16, 32):
        psi = statevector.trotter_evolve(psi0, hb, dims, T / steps, steps)
        errs.append(np.linalg.norm(psi - exact))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_fourth_order_composition_error_scales_as_dt4():
    # Suzuki's fourth-order composition of the symmetric step: global error
    # O(dt^4), so halving dt divides it by ~16; the coefficients sum to one
    # (a wrong s, a dropped sub-step or a wrong sign in 1 - 4s breaks both).
    sw = mps.step_sweeps(4)
    assert len(sw) == 15
    assert abs(sum(f for p, f in sw if p == 1) - 1.0) < 1e-15
    assert abs(sum(f for p, f in sw if p == 0) - 1.0) < 1e-15
    n, T = 6, 0.8
    dims, hb = models.tfim(n, 1.0, 1.0)
    H = models.full_hamiltonian(dims, hb)
    psi0 = statevector.product_vector(dims, [0] * n)
    exact = statevector.exact_evolve(psi0, H, T)
    errs = []
    for steps in (4, 8, 16):
        psi = statevector.trotter_evolve(psi0, hb, dims, T / steps, steps, order=4)
        errs.append(np.linalg.norm(psi - exact))
    assert 13.0 < errs[0] / errs[1] < 19.0 and 13.0 < errs[1] / errs[2] < 19.0
    # and it beats the second-order step at the same dt
    psi2 = statevector.trotter_evolve(psi0, hb, dims, T / 8, 8)
    assert errs[1] < 0.1 * np.linalg.norm(psi2 - exact)


def test_fourth_order_tebd_equals_its_state_vector_circuit():
    n, dt, steps = 8, 0.1, 4
    dims, hb = models.tfim(n, 1.0, 1.0)
    gates = {}

    def gfn(b, tau):
        if (b, tau) not in gates:
            gates[(b, tau)] = models.gate(hb[b], tau)
        return gates[(b, tau)]
    drv = mps.TEBD(mps.basis_product_state(dims, [0] * n), gfn, dt, 32, 0.0, method="full",
                   order=4)
    for _ in range(steps):
        drv.step()
    psi_sv = statevector.trotter_evolve(statevector.product_vector(dims, [0] * n), hb, dims, dt,
                                        steps, order=4)
    psi = mps.to_statevector(drv.mps)
    ov = abs(np.vdot(psi_sv, psi)) / (np.linalg.norm(psi_sv) * np.linalg.norm(psi))
    assert abs(1 - ov) < 1e-12
    assert drv.sweeps_done == 15 * steps


def test_full_hamiltonian_is_sum_of_bond_terms():
    # on-site split sums to one per site: compare with the chain H built directly
    n = 5
    dims, hb = models.tfim(n, 0.7, 1.3)
    H = models.full_hamiltonian(dims, hb)
    direct = np.zeros_like(H)
    for i in range(n):
        direct += -1.3 * np.kron(np.kron(np.eye(2 ** i), models.X), np.eye(2 ** (n - i - 1)))
    for b in range(n - 1):
        direct += -0.7 * np.kron(np.kron(np.eye(2 ** b), np.kron(models.Z, models.Z)),
                                 np.eye(2 ** (n - b - 2)))
    assert np.allclose(H, direct, atol=1e-14)


def test_free_fermion_matches_state_vector():
    n, dt, steps = 8, 0.05, 10
    J, h = wl.xx_couplings(n, seed=3)
    dims, hb = models.xx_field(J, h)
    lev = wl.neel_levels(n)
    psi = statevector.trotter_evolve(statevector.product_vector(dims, lev), hb, dims, dt, steps)
    zs = freefermion.z_profile(J, h, lev, dt, steps)
    for i in range(n):
        assert abs(statevector.local_expectation(psi, models.Z, i, dims).real - zs[i]) < 1e-12


def test_tebd_xx_chain_matches_free_fermions():
    n, dt, steps = 16, 0.02, 25
    J, h = wl.xx_couplings(n, seed=4)
    dims, hb = models.xx_field(J, h)
    lev = wl.neel_levels(n)
    m = mps.basis_product_state(dims, lev)
    zs = freefermion.z_profile(J, h, lev, dt, steps)
    # eps = 1e-20 per bond: the truncation error stays below 1e-10
    drv = mps.TEBD(m, lambda b, tau: models.gate(hb[b], tau), dt, 64, 1e-20, method="full")
    for _ in range(steps):
        drv.step()
    for i in range(n):
        assert abs(mps.expectation(drv.mps, models.Z, i).real - zs[i]) < 1e-10
    assert sum(x["w"] for x in drv.log) < 1e-17
    # eps = 1e-12: errors grow with the discarded weight but stay bounded by sqrt(sum w)
    m = mps.basis_product_state(dims, lev)
    drv = mps.TEBD(m, lambda b, tau: models.gate(hb[b], tau), dt, 64, 1e-12, method="full")
    for _ in range(steps):
        drv.step()
    sw = sum(x["w"] for x in drv.log)
    err = max(abs(mps.expectation(drv.mps, models.Z, i).real - zs[i]) for i in range(n))
    assert sw > 1e-12 and err < 10 * np.sqrt(sw)


def test_spin_boson_decoupled_spin_stays_put():
    # t0 = 0: the spin is decoupled and the chain stays in the vacuum.
    n, d = 6, 4
    dims, hb = models.spin_boson_chain(n, d, omega0=1.0, t0=0.0, omegas=1.0, hops=0.5)
    m = mps.basis_product_state(dims, [0] * n)
    drv = mps.TEBD(m, lambda b, tau: models.gate(hb[b], tau), 0.05, 20, 1e-10, method="full")
    for _ in range(10):
        drv.step()
    assert abs(mps.expectation(drv.mps, models.Z, 0).real - 1.0) < 1e-12
    assert all(c == 1 for c in drv.mps.chis())


def test_spin_boson_against_exact_diagonalisation():
    n, d, T = 4, 4, 0.6
    dims, hb = models.spin_boson_chain(n, d, omega0=1.0, t0=0.5, omegas=1.0, hops=0.5)
    H = models.full_hamiltonian(dims, hb)
    psi0 = statevector.product_vector(dims, [0] * n)
    exact = statevector.exact_evolve(psi0, H, T)
    z_exact = statevector.local_expectation(exact, models.Z, 0, dims).real
    errs = []
    for steps in (6, 12):
        m = mps.basis_product_state(dims, [0] * n)
        dt = T / steps
        drv = mps.TEBD(m, lambda b, tau: models.gate(hb[b], tau), dt, 64, 1e-14, method="rrsvd", seed=5)
        for _ in range(steps):
            drv.step()
        errs.append(abs(mps.expectation(drv.mps, models.Z, 0).real - z_exact))
    assert errs[1] < errs[0] and errs[1] < 2e-3
    # the spin-boson bond term is Hermitian and couples spin and first oscillator
    assert np.allclose(hb[0], hb[0].conj().T)


def test_truncation_bookkeeping_and_norm():
    # With truncation active, every renormalised update keeps unit norm, and the
    # discarded weight logged equals the squared tail of the Schmidt values.
    n = 10
    dims, hb, drv = _tfim_driver(n, 0.1, 4, 1e-6, "full")
    for _ in range(10):
        drv.step()
    assert abs(mps.norm2(drv.mps) - 1.0) < 1e-10
    ws = [x["w"] for x in drv.log]
    assert max(ws) > 0
    for x in drv.log:
        s = x["s"]
        assert len(s) == x["chi"] <= 4


def _embed(op, site, dims):
    left = int(np.prod(dims[:site]))
    right = int(np.prod(dims[site + 1:]))
    return np.kron(np.kron(np.eye(left), op), np.eye(right))


def test_spin_boson_hamiltonian_matches_second_quantised_form():
    # Eq. (H_1D) written with whole-chain operators, no bond split.
    n, d = 4, 3
    w0, t0, om, hop = 1.3, 0.4, 0.9, 0.6
    dims, hb = models.spin_boson_chain(n, d, omega0=w0, t0=t0, omegas=om, hops=hop)
    H = models.full_hamiltonian(dims, hb)
    b = [None] + [_embed(models.boson_annihilation(d), k, dims) for k in range(1, n)]
    direct = 0.5 * w0 * _embed(models.Z, 0, dims)
    direct = direct + t0 * _embed(models.X, 0, dims) @ (b[1] + b[1].conj().T)
    for k in range(1, n):
        direct = direct + om * b[k].conj().T @ b[k]
    for k in range(1, n - 1):
        direct = direct + hop * (b[k].conj().T @ b[k + 1] + b[k] @ b[k + 1].conj().T)
    assert np.allclose(H, direct, atol=1e-13)
    # truncated boson: [b, b^dag] = 1 except on the top level
    bb = models.boson_annihilation(d)
    comm = bb @ bb.conj().T - bb.conj().T @ bb
    assert np.allclose(np.diag(comm)[:-1], 1.0) and abs(comm[-1, -1] + (d - 1)) < 1e-12


def test_xx_hamiltonian_matches_direct_form():
    n = 4
    J, h = wl.xx_couplings(n, seed=9)
    dims, hb = models.xx_field(J, h)
    H = models.full_hamiltonian(dims, hb)
    direct = sum(h[i] * _embed(models.Z, i, dims) for i in range(n))
    for b in range(n - 1):
        direct = direct + 0.5 * J[b] * (_embed(models.X, b, dims) @ _embed(models.X, b + 1, dims)
                                        + _embed(models.Y, b, dims) @ _embed(models.Y, b + 1, dims))
    assert np.allclose(H, direct, atol=1e-13)


def test_gate_is_unitary_propagator():
    dims, hb = models.spin_boson_chain(3, 4)
    g = models.gate(hb[1], 0.1)
    assert np.allclose(g.conj().T @ g, np.eye(16), atol=1e-13)
    # first order in tau: G = 1 - i tau h + O(tau^2)
    tau = 1e-6
    g = models.gate(hb[1], tau)
    assert np.allclose((g - np.eye(16)) / tau, -1j * hb[1], atol=1e-4)


def test_adaptive_tebd_matches_fixed_rank_physics():
    # The adaptive-rank driver keeps every per-bond discarded weight <= eps and
    # follows the untruncated circuit as closely as the fixed-rank driver.
    n, dt, steps = 8, 0.05, 10
    dims, hb = models.tfim(n, 1.0, 1.0)
    res = {}
    for method in ("rrsvd", "rrsvd_adaptive"):
        m = mps.basis_product_state(dims, [0] * n)
        drv = mps.TEBD(m, lambda b, tau: models.gate(hb[b], tau), dt, 16, 1e-12, method=method, seed=3)
        for _ in range(steps):
            drv.step()
        assert max(x["w"] for x in drv.log) <= 1e-12
        res[method] = [mps.expectation(drv.mps, models.Z, i).real for i in range(n)]
    psi = statevector.trotter_evolve(statevector.product_vector(dims, [0] * n), hb, dims, dt, steps)
    zs = [statevector.local_expectation(psi, models.Z, i, dims).real for i in range(n)]
    for method in res:
        assert max(abs(a - b) for a, b in zip(res[method], zs)) < 1e-6
