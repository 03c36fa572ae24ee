"""Write the stored expected values under tests/golden/ (uses only oracle/).

tfim_n20_trotter.txt: <Z_i> after 100 symmetric Trotter steps (dt = 0.01,
T = 1) of the open transverse-field Ising chain, N = 20, J = h = 1, from
|0...0>, by the brute-force state vector of the same gate circuit (no
truncation).

xx_n40_gradient.txt: d<Z_0(T)>/dJ_b for the XX chain with random fields,
N = 40, J_b ~ U[0.8, 1.2], h_i ~ U[-1, 1] (seed 1504), Neel start, 50 steps of
dt = 0.02, chi_max = 64, relative discarded weight <= 1e-10 per bond: reverse
mode over the O-def run (full LAPACK SVD, every triplet coupled), central
finite differences (h = 1e-6) of the same run with its bond dimensions
replayed, and the truncation-free free-fermion closed form.

Usage: python tests/golden/make_golden.py [tfim|xx]
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import adjoint, freefermion, models, mps, statevector  # noqa: E402


def tfim_n20():
    n, dt, steps = 20, 0.01, 100
    dims, hb = models.tfim(n, 1.0, 1.0)
    psi = statevector.product_vector(dims, [0] * n)
    psi = statevector.trotter_evolve(psi, hb, dims, dt, steps)
    z = [statevector.local_expectation(psi, models.Z, i, dims).real for i in range(n)]
    with open(os.path.join(HERE, "tfim_n20_trotter.txt"), "w") as f:
        f.write("# <Z_i>(T=1) of the open TFIM, N=20, J=h=1, dt=0.01, 100 symmetric Trotter steps\n")
        f.write("# from |0...0>, untruncated state vector of the gate circuit (oracle/statevector.py)\n")
        f.write("# written by tests/golden/make_golden.py\n")
        for i, v in enumerate(z):
            f.write(f"{i} {v:.16e}\n")


def xx_n40_gradient():
    import workloads
    n, dt, steps, chi_max, eps = 40, 0.02, 50, 64, 1e-10
    couplings, fields = workloads.xx_couplings(n, seed=1504)
    hop = 0.5 * (np.kron(models.X, models.X) + np.kron(models.Y, models.Y))

    def gate_fn_of(jv):
        hb = models.xx_field(jv, fields)[1]
        cache = {}

        def g(b, tau):
            if (b, tau) not in cache:
                cache[(b, tau)] = models.gate(hb[b], tau)
            return cache[(b, tau)]
        return g
    dims, hb = models.xx_field(couplings, fields)
    levels = workloads.neel_levels(n)
    mps0 = mps.basis_product_state(dims, levels)
    val, grad, recs, _ = adjoint.tebd_gradient(
        mps0, gate_fn_of(couplings), lambda b: hb[b], lambda b, k: hop if b == k else None,
        n - 1, dt, steps, chi_max, eps, models.Z, 0)
    sched = [r["chi"] for r in recs]
    fd = adjoint.finite_difference_gradient(mps0, gate_fn_of, couplings, dt, steps, chi_max, eps,
                                            models.Z, 0, sched)
    ffg = freefermion.z_gradient(couplings, fields, levels, dt, steps)
    ffv = freefermion.z_profile(couplings, fields, levels, dt, steps)[0]
    with open(os.path.join(HERE, "xx_n40_gradient.txt"), "w") as f:
        f.write("# d<Z_0(T=1)>/dJ_b, XX chain + random fields, N=40, seed 1504, Neel start,\n")
        f.write("# 50 steps dt=0.02, chi_max=64, discarded weight <= 1e-10 per bond\n")
        f.write("# written by tests/golden/make_golden.py (oracle/adjoint.py, oracle/freefermion.py)\n")
        f.write(f"# value_tebd {val:.16e}\n")
        f.write(f"# value_free_fermion {ffv:.16e}\n")
        f.write(f"# max_chi {max(sched)}\n")
        f.write("# b J_b reverse_mode finite_difference free_fermion\n")
        for b in range(n - 1):
            f.write(f"{b} {couplings[b]:.16e} {grad[b]:.16e} {fd[b]:.16e} {ffg[b]:.16e}\n")


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("tfim", "all"):
        tfim_n20()
    if which in ("xx", "all"):
        xx_n40_gradient()
