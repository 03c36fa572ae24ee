"""Philox4x32-10 and the complex Gaussian test matrix (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper draws the n x l test matrix Omega with i.i.d. standard Gaussian
entries (Sec. IV, fixed-rank range finder; Alg. 1, first step) and notes that
the quality of the generator is immaterial.  To let a CPU run and a GPU run
use the *same* Omega without copying it, both sides implement the
counter-based generator Philox4x32-10 from its published definition
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11): ten rounds of the Philox S-box on a 128-bit counter with a 64-bit
key that is advanced by the Weyl constants between rounds.

Element (r, c) of Omega for stream (problem, call) uses counter
(r, c, problem, call) and key (seed low word, seed high word).  The first two
output words give two uniforms u = (x + 1/2) 2^-32 in (0, 1), and the
Box-Muller transform turns them into one complex standard normal
z = sqrt(-2 ln u1) exp(2 pi i u2) / sqrt(2), i.e. Re z, Im z ~ N(0, 1/2)
independently (a complex standard normal, E|z|^2 = 1).
"""
import numpy as np

# Constants of Philox4x32 (Salmon et al. 2011): round multipliers and the
# Weyl sequence increments applied to the key between rounds.
MULT0 = 0xD2511F53
MULT1 = 0xCD9E8D57
WEYL0 = 0x9E3779B9
WEYL1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF


def _mulhilo(a, b):
    """Full 64-bit product of two uint32 arrays, split into (hi, lo) words."""
    p = a.astype(np.uint64) * np.uint64(b)
    return (p >> np.uint64(32)).astype(np.uint64), (p & np.uint64(MASK32)).astype(np.uint64)


def philox4x32_10(counter, key):
    """Philox4x32 with 10 rounds.

    counter: array of shape (..., 4) of uint32 words (x0, x1, x2, x3).
    key:     pair (k0, k1) of uint32 words.
    Returns an array of shape (..., 4) of uint32 output words.

    One round maps (x0, x1, x2, x3) to
    (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0));
    the key is advanced by (W0, W1) before every round but the first.
    """
    c = np.asarray(counter, dtype=np.uint64) & np.uint64(MASK32)
    x0, x1, x2, x3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0 = np.uint64(int(key[0]) & MASK32)
    k1 = np.uint64(int(key[1]) & MASK32)
    for rnd in range(10):
        if rnd > 0:
            k0 = np.uint64((int(k0) + WEYL0) & MASK32)
            k1 = np.uint64((int(k1) + WEYL1) & MASK32)
        hi0, lo0 = _mulhilo(x0, MULT0)
        hi1, lo1 = _mulhilo(x2, MULT1)
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=-1).astype(np.uint32)


def uniform_open01(words):
    """Map uint32 words to doubles in (0, 1): u = (x + 1/2) * 2^-32."""
    return (np.asarray(words, dtype=np.float64) + 0.5) * (2.0 ** -32)


def gaussian_omega(n, l, seed, problem, call):
    """The n x l complex Gaussian test matrix for one RRSVD problem.

    Entry (r, c) is drawn from counter (r, c, problem, call) under key
    (seed & 0xffffffff, seed >> 32); see the module docstring.
    """
    seed = int(seed)
    key = (seed & MASK32, (seed >> 32) & MASK32)
    r = np.arange(n, dtype=np.uint64)[:, None] * np.ones((1, l), dtype=np.uint64)
    c = np.ones((n, 1), dtype=np.uint64) * np.arange(l, dtype=np.uint64)[None, :]
    ctr = np.stack([r, c,
                    np.full((n, l), int(problem) & MASK32, dtype=np.uint64),
                    np.full((n, l), int(call) & MASK32, dtype=np.uint64)], axis=-1)
    w = philox4x32_10(ctr, key)
    u1 = uniform_open01(w[..., 0])
    u2 = uniform_open01(w[..., 1])
    radius = np.sqrt(-2.0 * np.log(u1))
    angle = 2.0 * np.pi * u2
    return (radius * (np.cos(angle) + 1j * np.sin(angle)) / np.sqrt(2.0)).astype(np.complex128)
