"""Pins of the mixed-state (MPO) oracle: the Liouville-space bond
generators, gates and trace observables of oracle/mixed.py.

* Without jump operators an MPO of a pure state evolves as the pure state:
  the MPO TEBD of |0..0><0..0| must give the <Z_i> of the pure-state gate
  circuit (state vector) to 1e-12.
* A damped oscillator decays in closed form: with the coupling switched
  off, <n(t)> = n(0) exp(-kappa t) exactly, whatever dt.
* The Lindblad generator conserves the trace (the identity is a left null
  vector of every bond generator).
* Sharing each site's dissipator between its bonds is consistent: the
  Trotter circuit of a dissipative chain converges to exp(t L) with a
  second-order error (a wrong share leaves an O(1) error instead).
"""
import numpy as np

from oracle import mixed, models, mps, statevector


def _driver(dims, gens, dt, chi_max, eps, levels):
    ld = [d * d for d in dims]
    gates = {}

    def gfn(b, tau):
        if (b, tau) not in gates:
            gates[(b, tau)] = mixed.gate(gens[b], tau)
        return gates[(b, tau)]
    m = mps.basis_product_state(ld, [lv * d + lv for lv, d in zip(levels, dims)])
    return mps.TEBD(m, gfn, dt, chi_max, eps, method="full")


def test_unitary_mpo_tebd_equals_pure_state_circuit():
    n, dt, steps = 6, 0.05, 6
    dims, hb = models.tfim(n, 1.0, 1.0)
    gens = mixed.bond_generators(dims, hb, [[] for _ in range(n)])
    drv = _driver(dims, gens, dt, 256, 0.0, [0] * n)
    for _ in range(steps):
        drv.step()
    psi = statevector.trotter_evolve(statevector.product_vector(dims, [0] * n), hb, dims, dt, steps)
    for i in range(n):
        zm = mixed.trace_expectation(drv.mps, models.Z, i)
        zs = statevector.local_expectation(psi, models.Z, i, dims)
        assert abs(zm - zs) < 1e-12, (i, zm, zs)


def test_damped_oscillator_closed_form():
    d, kappa, dt, steps = 4, 0.3, 0.1, 10
    dims = [2, d]
    b = models.boson_annihilation(d)
    hb = models.bond_hamiltonians(dims, [np.zeros((2 * d, 2 * d))],
                                  [0.5 * models.Z, 1.0 * b.conj().T @ b])
    gens = mixed.bond_generators(dims, hb, [[], [np.sqrt(kappa) * b]])
    drv = _driver(dims, gens, dt, 16, 0.0, [0, 1])
    num = b.conj().T @ b
    for s in range(1, steps + 1):
        drv.step()
        t = s * dt
        assert abs(mixed.trace_expectation(drv.mps, num, 1) - np.exp(-kappa * t)) < 1e-12
        assert abs(mixed.trace_expectation(drv.mps, models.Z, 0) - 1.0) < 1e-12


def test_generators_conserve_the_trace():
    dims, hb = models.spin_boson_chain(3, 3, 1.0, 0.5, 1.0, 0.5)
    b = models.boson_annihilation(3)
    sm = np.array([[0, 0], [1, 0]], dtype=np.complex128)
    gens = mixed.bond_generators(dims, hb, [[0.2 * sm], [0.4 * b], [0.1 * b, 0.3 * b.conj().T @ b]])
    for g, (dl, dr) in zip(gens, [(2, 3), (3, 3)]):
        ident = np.kron(np.eye(dl).reshape(-1), np.eye(dr).reshape(-1))
        assert np.max(np.abs(ident @ g)) < 1e-13


def test_dissipative_trotter_circuit_converges_at_second_order():
    n, T = 3, 0.6
    dims, hb = models.tfim(n, 1.0, 0.7)
    sm = np.array([[0, 0], [1, 0]], dtype=np.complex128)
    gens = mixed.bond_generators(dims, hb, [[0.5 * sm] for _ in range(n)])
    Lfull = mixed.full_generator(dims, gens)
    ld = [d * d for d in dims]
    v0 = statevector.product_vector(ld, [0] * n)
    exact = scipy_expm_apply(Lfull, T, v0)
    errs = []
    for steps in (6, 12, 24):
        dt = T / steps
        v = v0.copy()
        for _ in range(steps):
            for parity, frac in mps.STEP_SWEEPS:
                for bnd in range(parity, n - 1, 2):
                    v = statevector.apply_two_site(v, mixed.gate(gens[bnd], frac * dt), bnd, ld)
        errs.append(np.linalg.norm(v - exact))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5
    # and the trace observable of the exact state is a valid expectation value
    z0 = mixed.vec_trace_expectation(exact, models.Z, 0, dims)
    assert abs(z0.imag) < 1e-12 and -1.0 <= z0.real <= 1.0


def scipy_expm_apply(L, t, v):
    import scipy.linalg
    return scipy.linalg.expm(t * L) @ v
