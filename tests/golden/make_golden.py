"""Write the stored expected values under tests/golden/ (uses only oracle/).

tfim_n20_trotter.txt: <Z_i> after 100 symmetric Trotter steps (dt = 0.01,
T = 1) of the open transverse-field Ising chain, N = 20, J = h = 1, from
|0...0>, by the brute-force state vector of the same gate circuit (no
truncation).  Usage: python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import models, statevector  # noqa: E402


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


if __name__ == "__main__":
    tfim_n20()
