"""CPU oracle for the TEBD two-site bond update with RRSVD truncation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or run anything under ``oracle/``; only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` do.  The oracle
shares no code with the HIP path: it has its own random-number generator
(``philox``), its own Hamiltonian and gate builders (``models``), its own
TEBD driver (``mps``) and its own linear algebra (``rrsvd``, built on
numpy/scipy LAPACK in float64 / complex128).

Modules (paper = Tamascelli, Rosenbach, Plenio, arXiv:1504.00992):

* ``philox``      -- Philox4x32-10 counter-based generator and the complex
                     Gaussian test matrix Omega of Sec. IV (Alg. 1, first step).
* ``rrsvd``       -- O-def: truncated SVD by full LAPACK gesvd (Sec. IV, best
                     rank-k approximation); O-alg: Alg. 1 followed by steps
                     i-iii of Sec. IV with a caller-supplied Omega; the
                     truncation rule built on the discarded weight of
                     Eq. (defdiscweigt) and the Frobenius identity of Sec. IV.
* ``mps``         -- Vidal-form MPS (Eq. defmps), Theta of Eq. (deftheta), the
                     gate update of Eq. (defupdatetheta), the blocked matrix of
                     Sec. II.B, lambda^-1 reabsorption, the symmetric
                     Suzuki-Trotter sweep order of Eq. (defst3rd), and exact
                     observables by transfer-matrix contraction.
* ``models``      -- TFIM, XX-plus-field and the chain-mapped spin-boson
                     Hamiltonian of Eq. (H_1D); two-site gates exp(-i tau h_b).
* ``statevector`` -- brute-force state vector of the same Trotter circuit and
                     exact diagonalisation (pins for the TEBD driver).
* ``freefermion`` -- exact single-particle propagation of the Trotterised XX
                     chain (Jordan-Wigner), a truncation-free pin.

Every function is written for clarity, not speed.  Each is pinned by a
``-m "not gpu"`` test against something other than itself (closed forms,
textbook identities, brute force, values printed in the paper).
"""
