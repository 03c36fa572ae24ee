"""GPU parity of rrsvd_truncate (HIP path) against the CPU oracle.

Tolerances (FP64 path): singular values |s_gpu - s_oracle| <= 1e-10 s_1
(normwise relative, the accuracy target of the FP64 path); discarded weight
within 1e-12 absolute (both sides evaluate the same Frobenius identity, so
they differ only by rounding of sums of O(1) numbers); chi' exact (integer
decision, test spectra keep their cuts away from ties); the rank-chi'
reconstructions U diag(S) V^H within 1e-10 s_1 entry-wise.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import philox, rrsvd as orr

pytestmark = pytest.mark.gpu

SEED = 1504


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1504_00992_amd import _lib
    _lib.load()


def _gpu(mats, chi_max, p, q, eps, seed=SEED, omegas=None, stream_id=0):
    from paper_1504_00992_amd import api
    As = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in mats]
    oms = None if omegas is None else [torch.from_numpy(o).cuda() for o in omegas]
    U, S, VH, chi, w, st = api.rrsvd_truncate(As, chi_max, p, q, eps, seed, stream_id, omegas=oms)
    torch.cuda.synchronize()
    return ([u.cpu().numpy() for u in U], [s.cpu().numpy() for s in S],
            [v.cpu().numpy() for v in VH], chi.cpu().numpy(), w.cpu().numpy(), st.cpu().numpy())


def _oracle(a, b, chi_max, p, q, eps, seed=SEED, stream_id=0, omega=None):
    m, n = a.shape
    l = orr.sketch_width(chi_max, p, m, n)
    om = philox.gaussian_omega(n, l, seed, b, stream_id) if omega is None else omega
    return orr.truncate_rrsvd(a, om, q, chi_max, eps)


def _compare(mats, res, chi_max, p, q, eps, omegas=None):
    U, S, VH, chi, w, st = res
    for b, a in enumerate(mats):
        ou, os_, ovh, ochi, ow, ost = _oracle(a, b, chi_max, p, q, eps,
                                             omega=None if omegas is None else omegas[b])
        s1 = max(os_[0], 1e-300)
        assert chi[b] == ochi, (b, chi[b], ochi)
        assert st[b] == ost, (b, st[b], ost)
        assert abs(w[b] - ow) <= 1e-12, (b, w[b], ow)
        c = ochi
        assert np.max(np.abs(S[b][:c] - os_)) <= 1e-10 * s1
        assert np.all(S[b][c:] == 0)
        rec_g = (U[b][:, :c] * S[b][None, :c]) @ VH[b][:c, :]
        rec_o = (ou * os_[None, :]) @ ovh
        assert np.max(np.abs(rec_g - rec_o)) <= 1e-10 * s1
        assert np.all(U[b][:, c:] == 0) and np.all(VH[b][c:, :] == 0)
        # orthonormal kept vectors (a zero singular value has no left vector)
        nz = S[b][:c] > 0
        u = U[b][:, :c][:, nz]
        assert np.allclose(u.conj().T @ u, np.eye(u.shape[1]), atol=1e-12)
        assert np.allclose(VH[b][:c] @ VH[b][:c].conj().T, np.eye(c), atol=1e-12)


# the QR size classes: (37, 53) register class 0; (190, 140, l = 33) and
# (300, 200, l = 20) register class 1 with a slot per reflector (16 and 32
# lanes per column); the 130-row side of (200, 130) register class 1 with
# alternating reflector buffers; (200, 200, l = 40) the LDS class on both
# sides; the larger ones the global class.  (300, 300, l = 66) also runs the
# small SVD's third class (C and J in LDS, 65 <= l <= 69).
@pytest.mark.parametrize("m,n,chi_max,p", [(37, 53, 8, 10), (190, 140, 23, 10), (300, 200, 10, 10),
                                           (200, 130, 40, 10), (130, 200, 40, 10),
                                           (300, 300, 50, 10), (700, 650, 64, 10),
                                           (200, 200, 30, 10), (300, 300, 56, 10)])
def test_parity_with_oracle_same_omega(m, n, chi_max, p):
    gen = wl.rng(m * 1000 + n)
    s = np.exp(-np.arange(min(m, n)) / (chi_max / 6.0))
    a = wl.known_spectrum(m, n, s, gen)
    res = _gpu([a], chi_max, p, 2, 1e-10)
    _compare([a], res, chi_max, p, 2, 1e-10)


def test_size_classes_of_the_parity_shapes():
    # the shapes above reach every factorisation kernel
    from paper_1504_00992_amd import _lib
    assert _lib.tebd_size_class(0, 37, 18) == 0
    assert _lib.tebd_size_class(0, 190, 33) == 1
    assert _lib.tebd_size_class(0, 200, 40) == 2
    assert _lib.tebd_size_class(0, 300, 60) == 3
    assert _lib.tebd_size_class(1, 0, 18) == 0
    assert _lib.tebd_size_class(1, 0, 40) == 1
    assert _lib.tebd_size_class(1, 0, 66) == 2
    assert _lib.tebd_size_class(1, 0, 74) == 3


def test_exact_when_sketch_covers_range():
    gen = wl.rng(5)
    s = np.exp(-np.arange(12) / 2.0)
    a = wl.known_spectrum(20, 12, s, gen)
    U, S, VH, chi, w, st = _gpu([a], 32, 10, 2, 1e-12)
    # l = min(42, 20, 12) = 12: exact SVD up to rounding (O-def)
    _, sd, _, cd, wd, _ = orr.truncate_full_svd(a, 32, 1e-12)
    assert chi[0] == cd
    assert np.max(np.abs(S[0][:cd] - sd)) < 1e-13
    assert abs(w[0] - wd) < 1e-13


def test_external_omega_and_q_values():
    gen = wl.rng(6)
    a = wl.known_spectrum(150, 120, np.exp(-np.arange(120) / 8.0), gen)
    for q in (0, 1, 3):
        l = orr.sketch_width(24, 6, 150, 120)
        om = philox.gaussian_omega(120, l, 99, 7, 3) * (1 + 0.5j)
        res = _gpu([a], 24, 6, q, 1e-8, omegas=[om])
        _compare([a], res, 24, 6, q, 1e-8, omegas=[om])


def test_batched_heterogeneous_sizes_and_edge_cases():
    gen = wl.rng(7)
    mats = [
        wl.known_spectrum(256, 256, wl.exp_spectrum(256), gen),        # cfg-like spectrum
        wl.known_spectrum(33, 97, np.exp(-np.arange(33) / 3.0), gen),  # ragged, wide
        wl.known_spectrum(64, 64, np.array([1.0, .7, .3, .1, .01]), gen),  # rank 5
        np.zeros((16, 9), dtype=np.complex128),                        # zero matrix
        wl.ginibre(1, 10, gen),                                        # one row
        wl.ginibre(10, 1, gen),                                        # one column
        wl.known_spectrum(80, 80, np.linspace(1, 0.5, 80), gen),       # flat: chi_max binds
    ]
    res = _gpu(mats, 16, 10, 2, 1e-10)
    _compare(mats, res, 16, 10, 2, 1e-10)
    U, S, VH, chi, w, st = res
    assert chi[2] == 5 and w[2] < 1e-14
    assert chi[3] == 1 and S[3][0] == 0 and w[3] == 0
    assert chi[4] == 1 and chi[5] == 1
    assert chi[6] == 16 and st[6] == orr.STATUS_CHI_BOUND


def test_fixed_rank_mode():
    gen = wl.rng(8)
    a = wl.known_spectrum(90, 70, np.exp(-np.arange(70) / 5.0), gen)
    res = _gpu([a], 12, 8, 2, 0.0)
    _compare([a], res, 12, 8, 2, 0.0)
    assert res[3][0] == 12


def test_batched_workload_full_size_sampled():
    # The 256-matrix workload at full size (sizes 256..2048) in one launch;
    # one problem of each size is recomputed by the oracle.
    from paper_1504_00992_amd import api
    sizes = wl.batched_rrsvd_sizes()
    mats = wl.batched_rrsvd_matrices_device(sizes)
    U, S, VH, chi, w, st = api.rrsvd_truncate(mats, 64, 10, 2, 1e-10, SEED, 0)
    torch.cuda.synchronize()
    S = [s.cpu().numpy() for s in S]
    chi, w, st = chi.cpu().numpy(), w.cpu().numpy(), st.cpu().numpy()
    picked = {}
    for i, n in enumerate(sizes):
        picked.setdefault(n, i)
    for n, i in sorted(picked.items()):
        a = mats[i].cpu().numpy()
        ou, os_, ovh, ochi, ow, ost = _oracle(a, i, 64, 10, 2, 1e-10)
        assert chi[i] == ochi == 64 and st[i] == ost == orr.STATUS_CHI_BOUND
        assert abs(w[i] - ow) <= 1e-12
        assert np.max(np.abs(S[i][:64] - os_)) <= 1e-10
        rec_g = (U[i][:, :64].cpu().numpy() * S[i][None, :64]) @ VH[i][:64].cpu().numpy()
        assert np.max(np.abs(rec_g - (ou * os_[None, :]) @ ovh)) <= 1e-10
    # properties at every problem: sorted values, Ritz bound s_hat_j <= s_j,
    # leading values close to the exact spectrum (approximation quality of
    # RRSVD with k = 64, p = 10, q = 2 on s_i = exp(-i/25), not a parity check)
    for i, n in enumerate(sizes):
        s_true = wl.exp_spectrum(n)[:64]
        assert np.all(np.diff(S[i][:64]) <= 1e-15)
        assert np.all(S[i][:64] <= s_true + 1e-12)
        assert np.max(np.abs(S[i][:12] - s_true[:12])) < 1e-10
        assert np.max(np.abs(S[i][:64] - s_true)) < 1e-2


@pytest.mark.parametrize("n", [900, 4900])
def test_table_two_shapes_match_oracle(n):
    # The mixed-state Theta shapes of the paper's timing table (d^2 chi with
    # chi = 100: 900 ... 4900) at k = p = 100, q = 2 (l = 200).  n = 4900
    # runs the global-memory QR with its reflectors in the slab (rows beyond
    # the LDS budget).  Rank-300 known spectrum s_i = exp(-i/30).
    from paper_1504_00992_amd import _lib
    assert _lib.tebd_size_class(0, n, 200) == 3
    gen = wl.rng(n + 3)
    a = wl.known_spectrum(n, n, np.exp(-np.arange(300) / 30.0), gen)
    res = _gpu([a], 100, 100, 2, 1e-10)
    _compare([a], res, 100, 100, 2, 1e-10)


def test_wide_sketch_tiles_give_the_same_results():
    # the autotune cache's tile variants of the sketch, power-iteration and
    # projection products: all agree with the oracle; 32 x 32 and 64 x 64
    # tiles with each other exactly (the K order of every output element is
    # the same), the split-depth 16 x 16 tiles to rounding
    from paper_1504_00992_amd import _lib
    gen = wl.rng(31)
    shapes = [(300, 200), (700, 650), (64, 90)]
    mats = [wl.known_spectrum(m, n, np.exp(-np.arange(min(m, n)) / 9.0), gen) for m, n in shapes]
    outs = []
    try:
        for v in (0, 1, 2):
            assert _lib.tebd_tune_set(0, 700, 74, v) == 0
            res = _gpu(mats, 64, 10, 2, 1e-10)
            _compare(mats, res, 64, 10, 2, 1e-10)
            outs.append(res)
    finally:
        _lib.tebd_tune_set(0, 700, 74, -1)
    for o in outs[1:]:
        for b in range(len(mats)):
            assert outs[0][3][b] == o[3][b]
            assert np.max(np.abs(outs[0][1][b] - o[1][b])) <= 1e-13 * outs[0][1][b][0]


def test_autotuner_times_every_variant(tmp_path):
    from paper_1504_00992_amd import _lib, autotune
    path = str(tmp_path / "tune.json")
    try:
        entries = autotune.tune(buckets=((256, 64),), batch=4, reps=1, path=path)
        assert len(entries) == 1 and entries[0]["variant"] in autotune.VARIANTS
        assert len(entries[0]["sketch_ms"]) == len(autotune.VARIANTS)
        assert all(ms > 0 for ms in entries[0]["sketch_ms"])
        assert _lib.tebd_tune_get(0, 256, 64) == entries[0]["variant"]
        _lib.tebd_tune_set(0, 256, 64, -1)
        assert autotune.load(path)[0]["variant"] == entries[0]["variant"]
    finally:
        _lib.tebd_tune_set(0, 256, 64, -1)


def test_workload_tuning_sets_its_buckets_and_keeps_the_others(tmp_path):
    # tune_workload: every variant timed on the given run, the fastest stored
    # for all its buckets, merged into an existing cache file
    import json
    import torch
    from paper_1504_00992_amd import _lib, autotune
    path = str(tmp_path / "tune.json")
    autotune.save([{"precision": 0, "rows": 2048, "width": 128, "variant": 1},
                   {"precision": 0, "rows": 256, "width": 64, "variant": 0}], path)
    gen = wl.rng(5)
    mats = [wl.known_spectrum(200, 180, np.exp(-np.arange(180) / 12.0), gen) for _ in range(3)]
    calls = []

    def run():
        calls.append(1)
        _gpu(mats, 24, 10, 2, 1e-10)
        torch.cuda.synchronize()
    buckets = ((256, 32), (256, 64))
    try:
        entries = autotune.tune_workload(run, "test_batch", buckets=buckets, reps=1, path=path)
        assert len(calls) == 2 * len(autotune.VARIANTS)   # a warm-up and one timed run each
        best = entries[0]["variant"]
        assert best in autotune.VARIANTS and all(e["variant"] == best for e in entries)
        assert len(entries[0]["workload_s"]) == len(autotune.VARIANTS)
        assert _lib.tebd_tune_get(0, 256, 64) == best and _lib.tebd_tune_get(0, 200, 20) == best
        with open(path) as f:
            stored = {(e["rows"], e["width"]): e for e in json.load(f)["entries"]}
        assert stored[(2048, 128)]["variant"] == 1                 # other buckets kept
        assert stored[(256, 64)]["variant"] == best and stored[(256, 64)]["workload"] == "test_batch"
        assert len(stored) == 3
    finally:
        for r, w in buckets:
            _lib.tebd_tune_set(0, r, w, -1)


def test_gram_qr_falls_back_on_a_rank_deficient_sketch():
    # A 300 x 300 matrix of rank 20 with l = 60: the QRs of this size go to
    # the Gram-based path first; the first sketch is rank deficient, so its
    # Cholesky refuses (TEBD_DEV_QR_FALLBACK) and the pivoted Householder
    # QR reveals the rank; the power iterations' QRs of the rank-20 bases
    # then pass.  Results as the oracle's.
    from paper_1504_00992_amd import _lib
    assert _lib.tebd_size_class(0, 300, 60) >= 2
    gen = wl.rng(41)
    a = wl.known_spectrum(300, 300, np.exp(-np.arange(20) / 3.0), gen)
    U, S, VH, chi, w, st = _gpu([a], 50, 10, 2, 1e-10)
    assert st[0] & _lib.DEV_QR_FALLBACK
    _compare([a], (U, S, VH, chi, w, st & ~_lib.DEV_QR_FALLBACK), 50, 10, 2, 1e-10)
