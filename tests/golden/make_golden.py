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

spin_boson_n100_adaptive.txt: the 16-chain spin-boson workload (N = 100,
spin-1/2 then 99 oscillators truncated at d = 10, t_n = 0.5, omega_n = 1,
dt = 0.05, chi_max = 100, p = 10, q = 2, relative discarded weight <= 1e-10
per bond, two-stage adaptive rank, Philox seed 1504), chains 0 and 15, by the
oracle's step-by-step RRSVD TEBD: bond dimensions, <sigma_z> of the spin and
<n_i> of oscillators 1, 2, 5, 10, 20 after 50, 100, 150 and 200 steps, and
every lambda after 200 steps.  Also the smallest relative distance of a
truncation decision from the threshold over the run (near-ties, where two
correct runs may cut differently).

spin_boson_n100_chi128.txt: chain 0 of the same workload at chi_max = 128
(the mixed-precision comparison): <sigma_z> of the spin after 50, 100, 150
and 200 steps and every lambda after 200 steps, FP64 oracle.

Usage: python tests/golden/make_golden.py [tfim|xx|spinboson|chi128]
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


SB_CHAINS = (0, 15)
SB_CHECK_STEPS = (50, 100, 150, 200)
SB_SITES = (1, 2, 5, 10, 20)


def spin_boson_n100():
    n, d, dt, steps, chi_max, eps = 100, 10, 0.05, 200, 100, 1e-10
    dims, hb = models.spin_boson_chain(n, d, 1.0, 0.5, 1.0, 0.5)
    cache = {}

    def gfn(b, tau):
        if (b, tau) not in cache:
            cache[(b, tau)] = models.gate(hb[b], tau)
        return cache[(b, tau)]
    num = np.diag(np.arange(d)).astype(np.complex128)
    out = []
    for chain in SB_CHAINS:
        drv = mps.TEBD(mps.basis_product_state(dims, [0] * n), gfn, dt, chi_max, eps,
                       method="rrsvd_adaptive", p=10, q=2, seed=1504, chain=chain)
        rows = []
        for s in range(1, steps + 1):
            drv.step()
            if s in SB_CHECK_STEPS:
                obs = [mps.expectation(drv.mps, models.Z, 0).real]
                obs += [mps.expectation(drv.mps, num, i).real for i in SB_SITES]
                rows.append((s, drv.mps.chis(), obs))
        margin = np.inf
        for info in drv.log:
            sv, f2, c = info["s"], info["frob2"], info["chi"]
            if f2 <= 0:
                continue
            w = 1.0 - np.cumsum(sv ** 2) / f2
            for k in (c - 2, c - 1):  # w(c - 1) and w(c), 0-based
                if 0 <= k < len(w):
                    margin = min(margin, abs(w[k] - eps) / eps)
        out.append((chain, rows, [l.copy() for l in drv.mps.lambdas], margin))
    with open(os.path.join(HERE, "spin_boson_n100_adaptive.txt"), "w") as f:
        f.write("# spin-boson chain N=100 (spin + 99 oscillators, d=10), t_n=0.5, w_n=1, dt=0.05,\n")
        f.write("# chi_max=100, RRSVD p=10 q=2, w<=1e-10 per bond, two-stage adaptive rank, seed 1504\n")
        f.write("# written by tests/golden/make_golden.py (oracle/mps.py, method rrsvd_adaptive)\n")
        f.write("# obs lines: chain step <sigma_z_0> <n_1> <n_2> <n_5> <n_10> <n_20>\n")
        f.write("# chi lines: chain step chi_0 .. chi_N;  lam lines: chain bond lambda_1 ..\n")
        for chain, rows, lams, margin in out:
            f.write(f"margin {chain} {margin:.6e}\n")
            for s, chis, obs in rows:
                f.write(f"obs {chain} {s} " + " ".join(f"{v:.16e}" for v in obs) + "\n")
                f.write(f"chi {chain} {s} " + " ".join(str(c) for c in chis) + "\n")
            for b, lam in enumerate(lams):
                f.write(f"lam {chain} {b} " + " ".join(f"{v:.16e}" for v in lam) + "\n")


def spin_boson_n100_chi128():
    n, d, dt, steps, chi_max, eps = 100, 10, 0.05, 200, 128, 1e-10
    dims, hb = models.spin_boson_chain(n, d, 1.0, 0.5, 1.0, 0.5)
    cache = {}

    def gfn(b, tau):
        if (b, tau) not in cache:
            cache[(b, tau)] = models.gate(hb[b], tau)
        return cache[(b, tau)]
    drv = mps.TEBD(mps.basis_product_state(dims, [0] * n), gfn, dt, chi_max, eps,
                   method="rrsvd_adaptive", p=10, q=2, seed=1504, chain=0)
    z = []
    for s in range(1, steps + 1):
        drv.step()
        if s % 50 == 0:
            z.append((s, mps.expectation(drv.mps, models.Z, 0).real))
    with open(os.path.join(HERE, "spin_boson_n100_chi128.txt"), "w") as f:
        f.write("# spin-boson chain N=100 (spin + 99 oscillators, d=10), t_n=0.5, w_n=1, dt=0.05,\n")
        f.write("# chi_max=128, RRSVD p=10 q=2, w<=1e-10 per bond, two-stage adaptive rank, seed 1504,\n")
        f.write("# chain 0; written by tests/golden/make_golden.py (oracle/mps.py, FP64)\n")
        f.write("# obs lines: step <sigma_z_0>;  lam lines: bond lambda_1 .. (after 200 steps)\n")
        for s, v in z:
            f.write(f"obs {s} {v:.16e}\n")
        for b, lam in enumerate(drv.mps.lambdas):
            f.write(f"lam {b} " + " ".join(f"{v:.16e}" for v in lam) + "\n")


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("tfim", "all"):
        tfim_n20()
    if which in ("xx", "all"):
        xx_n40_gradient()
    if which in ("spinboson", "all"):
        spin_boson_n100()
    if which in ("chi128", "all"):
        spin_boson_n100_chi128()
