"""Truncated SVD by definition (O-def) and by RRSVD step by step (O-alg).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

All arithmetic is complex128 / float64 on the CPU through numpy and scipy's
LAPACK.  No blocking, fusion or reordering beyond what the definitions state.

Paper: Tamascelli, Rosenbach, Plenio, arXiv:1504.00992.
"""
import numpy as np
import scipy.linalg

# Per-problem status bits (same meaning on both sides; the values are part of
# the published C interface, restated here so the oracle needs no header).
STATUS_CHI_BOUND = 16


def lapack_svd(a):
    """Thin SVD by LAPACK's gesvd; singular values sorted descending.

    Sec. IV: A = U Sigma V^H with sigma_1 >= sigma_2 >= ...
    """
    u, s, vh = scipy.linalg.svd(np.asarray(a, dtype=np.complex128),
                                full_matrices=False, lapack_driver="gesvd")
    return u, s, vh


def truncation_rank(weights, chi_max, eps):
    """Bond dimension kept after truncation, its discarded weight, status.

    weights[c-1] = w(c), the relative discarded weight of keeping the first c
    singular values (Sec. II.C, Eq. defdiscweigt, divided by ||A||_F^2).
    Rule: chi' = min(chi_max, smallest c >= 1 with w(c) <= eps), c ranging
    over the available values.  eps <= 0 means fixed rank
    chi' = min(chi_max, len(weights)).  Returns (chi', w(chi'), status) with
    status = STATUS_CHI_BOUND when no c <= chi_max meets a positive eps.
    """
    w = np.asarray(weights, dtype=np.float64)
    cap = min(int(chi_max), len(w))
    if eps <= 0.0:
        return cap, float(max(w[cap - 1], 0.0)), 0
    ok = np.nonzero(w <= eps)[0]
    if len(ok) and ok[0] + 1 <= cap:
        c = int(ok[0]) + 1
        return c, float(max(w[c - 1], 0.0)), 0
    return cap, float(max(w[cap - 1], 0.0)), STATUS_CHI_BOUND


def tail_weights(sig):
    """w(c) = sum_{j>c} sigma_j^2 / sum_j sigma_j^2 (the plain definition)."""
    s2 = np.asarray(sig, dtype=np.float64) ** 2
    total = np.sum(s2)
    if total <= 0.0:
        return np.zeros(len(s2))
    tails = np.array([np.sum(s2[c:]) for c in range(1, len(s2) + 1)])
    return tails / total


def frobenius_weights(sig, frob2):
    """w(c) = (||A||_F^2 - sum_{j<=c} sigma_j^2) / ||A||_F^2.

    The Frobenius-norm identity of Sec. IV (||(I - QQ^H)A||_F^2 =
    ||A||_F^2 - ||Q^H A||_F^2, with Q the kept left singular vectors) turns
    the l values an RRSVD returns, plus ||A||_F^2 from the entries of A,
    into the discarded weight of every rank c <= l.
    """
    s2 = np.asarray(sig, dtype=np.float64) ** 2
    if frob2 <= 0.0:
        return np.zeros(len(s2))
    return (frob2 - np.cumsum(s2)) / frob2


def truncate_full_svd(a, chi_max, eps):
    """O-def: best rank-chi' factors of A from a full LAPACK SVD.

    Sec. IV: keep the chi' largest singular triplets (Eckart-Young).  The
    discarded weight is the plain definition sum_{j>chi'} sigma_j^2 divided
    by ||A||_F^2 = sum_j sigma_j^2.
    Returns (U[:, :chi'], s[:chi'], Vh[:chi', :], chi', w, status).
    """
    u, s, vh = lapack_svd(a)
    chi, w, status = truncation_rank(tail_weights(s), chi_max, eps)
    return u[:, :chi], s[:chi], vh[:chi, :], chi, w, status


def sketch_width(k, p, m, n):
    """l = min(k + p, m, n): Alg. 1 needs l columns, at most the rank bound."""
    return int(min(k + p, m, n))


RANK_TOL = 1e-13


def range_basis(y, tol=RANK_TOL):
    """Orthonormal basis of the numerical range of Y (the QR steps of Alg. 1).

    Householder QR with column pivoting (LAPACK geqp3), Y P = Q R with
    |R_00| >= |R_11| >= ...; the basis keeps the r leading columns of Q with
    |R_jj| > tol |R_00| (r >= 1).  For a well-conditioned Y this is span(Y);
    for a numerically rank-deficient sketch it drops the directions that
    carry no information about A.  The paper leaves the QR method open.
    """
    q, r, _ = scipy.linalg.qr(np.asarray(y, dtype=np.complex128), mode="economic", pivoting=True)
    d = np.abs(np.diag(r))
    if len(d) == 0:
        return q
    keep = max(1, int(np.sum(d > tol * d[0])))
    return q[:, :keep]


def orthonormal_basis(y):
    """Q of the plain Householder QR Y = Q R (LAPACK geqrf/ungqr), every column.

    Used for the QRs of the power iterations, whose inputs A^H Q and A Qt
    have the rank r that the first QR kept (in exact arithmetic).
    """
    q, _ = scipy.linalg.qr(np.asarray(y, dtype=np.complex128), mode="economic")
    return q


def rrsvd_range(a, omega, q):
    """Alg. 1 (randomized range finder with q power iterations).

    Y0 = A Omega, Y0 = Q0 R0; for j = 1..q: Yt_j = A^H Q_{j-1} = Qt_j Rt_j,
    Y_j = A Qt_j = Q_j R_j.  The first QR reveals the numerical rank r <= l
    (range_basis); the power iterations orthonormalise their r columns
    (orthonormal_basis).  Returns Q_q (m x r, orthonormal columns).
    """
    a = np.asarray(a, dtype=np.complex128)
    y = a @ omega
    qmat = range_basis(y)
    for _ in range(q):
        yt = a.conj().T @ qmat
        qt = orthonormal_basis(yt)
        y = a @ qt
        qmat = orthonormal_basis(y)
    return qmat


def rrsvd(a, omega, q):
    """Alg. 1 followed by steps i-iii of Sec. IV.

    i) B = Q^H A;  ii) B = Ut Sigma V^H (LAPACK gesvd);  iii) U = Q Ut.
    Returns (U, s, Vh) with r <= l = omega.shape[1] triplets (r: the
    numerical rank kept by the range finder).
    """
    a = np.asarray(a, dtype=np.complex128)
    qmat = rrsvd_range(a, omega, q)
    b = qmat.conj().T @ a
    ut, s, vh = lapack_svd(b)
    return qmat @ ut, s, vh


def first_stage_rank(chi_mid, chi_max):
    """Target rank of the first stage of the adaptive scheme.

    The bond dimension before the update plus a margin of max(4, chi_mid/4)
    (rounded up), capped by chi_max.  A bond whose new dimension exceeds it
    takes the second stage; in TEBD steps of a small time step the bond
    dimension grows by a few per update at most.
    """
    return int(min(chi_max, chi_mid + max(4, (chi_mid + 3) // 4)))


def adaptive_factors(a, omega_of, q, chi_max, eps, k1, p):
    """Two-stage adaptive-rank RRSVD (TEBD with a tolerance), all factors.

    This two-stage rule is this project's own design, not the paper's
    Accuracy Check (Sec. IV, Alg. 2 grows Q by r probe columns until its
    estimated range error meets the tolerance; see ``accuracy_check``).  It
    uses the exact residual ||(I - QQ^H)A||_F that the Frobenius identity of
    Sec. IV gives from the factors.  Stage 1 runs the RRSVD with l1 = min(k1 + p, m, n) and is
    accepted when some c <= k1 has relative discarded weight w(c) <= eps
    (w from the Frobenius identity, so the bound is exact for the factors
    returned).  Otherwise stage 2 repeats with the fixed-rank width
    l2 = min(chi_max + p, m, n).  omega_of(l) returns the n x l test matrix;
    the first l1 columns of the stage-2 matrix are those of stage 1.
    Returns (U, s, Vh, chi', w, status, stage) with every triplet of the
    accepted stage (chi' of them are kept) and stage = 1 or 2.
    """
    a = np.asarray(a, dtype=np.complex128)
    m, n = a.shape
    l1 = sketch_width(k1, p, m, n)
    l2 = sketch_width(chi_max, p, m, n)
    u, s, vh = rrsvd(a, omega_of(l1), q)
    frob2 = float(np.vdot(a, a).real)
    wts = frobenius_weights(s, frob2)
    if l1 >= l2:
        chi, w, status = truncation_rank(wts, chi_max, eps)
        return u, s, vh, chi, w, status, 1
    chi, w, status = truncation_rank(wts, min(k1, chi_max), eps)
    if status == 0 and eps > 0.0:
        return u, s, vh, chi, w, status, 1
    u, s, vh = rrsvd(a, omega_of(l2), q)
    chi, w, status = truncation_rank(frobenius_weights(s, frob2), chi_max, eps)
    return u, s, vh, chi, w, status, 2


def truncate_rrsvd_adaptive(a, omega_of, q, chi_max, eps, k1, p):
    """``adaptive_factors`` cut to the kept triplets.

    Returns (U[:, :chi'], s[:chi'], Vh[:chi', :], chi', w, status, stage).
    """
    u, s, vh, chi, w, status, stage = adaptive_factors(a, omega_of, q, chi_max, eps, k1, p)
    return u[:, :chi], s[:chi], vh[:chi, :], chi, w, status, stage


def truncate_rrsvd(a, omega, q, chi_max, eps):
    """O-alg: RRSVD with the given Omega, then the truncation rule.

    The discarded weight uses the Frobenius identity of Sec. IV with
    ||A||_F^2 taken from the entries of A (the RRSVD only sees l values).
    Returns (U[:, :chi'], s[:chi'], Vh[:chi', :], chi', w, status).
    """
    a = np.asarray(a, dtype=np.complex128)
    u, s, vh = rrsvd(a, omega, q)
    frob2 = float(np.vdot(a, a).real)
    chi, w, status = truncation_rank(frobenius_weights(s, frob2), chi_max, eps)
    return u[:, :chi], s[:chi], vh[:chi, :], chi, w, status


# ---------------------------------------------------------------------------
# Accuracy Check (Sec. IV, Theorem 2, Alg. 2, Fact 1).
#
# Theorem 2: for M = (I - QQ^H) A and r standard Gaussian vectors w_i,
#   P( ||M|| <= 10 sqrt(2/pi) max_i ||M w_i|| ) >= 1 - 10^-r.
# Fact 1: if sigma_j <= sigma_1 / j then ||A||_F <= (pi / sqrt 6) ||A||.
# Together (the paper's combination, with the larger of its two printed
# constants, (10/3) pi >= 10 sqrt(pi/3)) the Frobenius residual is bounded
# by ACC_CONST max_i ||M w_i|| with probability 1 - 10^-r.

THEOREM2_CONST = 10.0 * np.sqrt(2.0 / np.pi)
FACT1_CONST = np.pi / np.sqrt(6.0)
ACC_CONST = 10.0 * np.pi / 3.0


def probe_residual(a, qmat, omega_r):
    """max_i ||(I - QQ^H) A w_i|| over the columns w_i of omega_r (and B = A Omega_r)."""
    b = np.asarray(a, dtype=np.complex128) @ omega_r
    d = b - qmat @ (qmat.conj().T @ b)
    return float(np.max(np.linalg.norm(d, axis=0))), b


def accuracy_check(a, qmat, r, tol, probe_of, l_cap, col0):
    """Alg. 2: grow the basis Q by blocks of r Gaussian probes.

    Each round draws Omega_r (n x r, columns col0, col0 + 1, ... of the test
    stream: probe_of(c0, r)), forms B = A Omega_r and D = (I - QQ^H) B and
    MAX = max_i ||d_i||.  When MAX > tol, Q becomes the Q factor of [Q | B]
    (l grows by r).  The loop repeats while MAX > tol and l <= n - r.  The
    basis never passes the capacity l_cap (a workspace bound, not in the
    paper): a block that would is cut to the columns that still fit, and
    when none fits the loop stops (returned as capped).  Returns (Q, rounds,
    capped, history of MAX).
    """
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[1]
    l = qmat.shape[1]
    rounds = 0
    capped = False
    hist = []
    c0 = col0
    while True:
        mx, b = probe_residual(a, qmat, probe_of(c0, r))
        c0 += r
        hist.append(mx)
        if mx > tol:
            w = min(r, l_cap - l)  # the last block fills the capacity
            if w <= 0:
                capped = True
                break
            qmat = orthonormal_basis(np.hstack([qmat, b[:, :w]]))
            l += w
            rounds += 1
        if not (mx > tol and l <= n - r):
            break
    return qmat, rounds, capped, hist


def rrsvd_accuracy(a, probe_of, q, k0, p, r, eps, l_cap):
    """RRSVD with the Accuracy Check, step by step.

    Alg. 1's first three steps with l0 = min(k0 + p, m, n) columns (Y0 =
    A Omega, the rank-revealing QR), then Alg. 2 with probes of r columns
    and tol = sqrt(eps) ||A||_F / ACC_CONST (eps: the relative discarded
    weight, so the Frobenius residual is sqrt(eps) ||A||_F), then the q power
    iterations of Alg. 1 on the grown basis and steps i-iii.  probe_of(c0, w)
    returns columns c0 .. c0 + w - 1 of the Gaussian stream (the first l0
    are Omega).  Returns (U, s, Vh, rounds, capped).
    """
    a = np.asarray(a, dtype=np.complex128)
    m, n = a.shape
    l0 = sketch_width(k0, p, m, n)
    qmat = range_basis(a @ probe_of(0, l0))
    frob = float(np.sqrt(np.vdot(a, a).real))
    tol = np.sqrt(max(eps, 0.0)) * frob / ACC_CONST
    qmat, rounds, capped, _ = accuracy_check(a, qmat, r, tol, probe_of, min(l_cap, m, n), l0)
    for _ in range(q):
        qt = orthonormal_basis(a.conj().T @ qmat)
        qmat = orthonormal_basis(a @ qt)
    b = qmat.conj().T @ a
    ut, s, vh = lapack_svd(b)
    return qmat @ ut, s, vh, rounds, capped


def truncate_rrsvd_accuracy(a, probe_of, q, chi_max, eps, k0, p, r):
    """``rrsvd_accuracy`` (capacity chi_max + p) and the truncation rule.

    Returns (U[:, :chi'], s[:chi'], Vh[:chi', :], chi', w, status, rounds).
    """
    a = np.asarray(a, dtype=np.complex128)
    u, s, vh, rounds, capped = rrsvd_accuracy(a, probe_of, q, k0, p, r, eps, chi_max + p)
    frob2 = float(np.vdot(a, a).real)
    chi, w, status = truncation_rank(frobenius_weights(s, frob2), chi_max, eps)
    return u[:, :chi], s[:chi], vh[:chi, :], chi, w, status, rounds
