"""rrsvd_truncate_noalloc (static scratch, no workspace) against
rrsvd_truncate (caller workspace) through the C interface.

Both run the same kernels on the same inputs and the same Philox test
matrices, so chi', the status bits and the discarded weights must agree
exactly and the singular values and rank-chi' reconstructions to 1e-10 s_1
(the FP64 parity bar).  Two calls in a row, the second with a smaller batch,
check that the shared scratch carries nothing from one call to the next.
"""
import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu
SEED = 1504


def _mats(shapes, seed):
    gen = wl.rng(seed)
    out = []
    for m, n in shapes:
        r = min(m, n)
        a = wl.known_spectrum(m, n, np.exp(-np.arange(r) / 6.0), gen)
        out.append(torch.from_numpy(a).cuda())
    return out


def _run(mats, chi_max, p, q, eps, noalloc, stream_id):
    from paper_1504_00992_amd import _lib, api
    dev = mats[0].device
    m = [a.shape[0] for a in mats]
    n = [a.shape[1] for a in mats]
    nmax = max(n)
    U = [torch.full((mi, chi_max), 7.0 + 0j, dtype=torch.complex128, device=dev) for mi in m]
    S = [torch.full((chi_max,), 7.0, dtype=torch.float64, device=dev) for _ in mats]
    VH = [torch.full((chi_max, nmax), 7.0 + 0j, dtype=torch.complex128, device=dev) for _ in mats]
    chi = torch.full((len(mats),), -1, dtype=torch.int32, device=dev)
    w = torch.full((len(mats),), -1.0, dtype=torch.float64, device=dev)
    st = torch.full((len(mats),), -1, dtype=torch.int32, device=dev)
    prm = _lib.params(chi_max, p, q, eps, 1e-14, SEED, stream_id)
    args = (m, n, [a.data_ptr() for a in mats], [a.stride(0) for a in mats], None, prm,
            [u.data_ptr() for u in U], chi_max, [s.data_ptr() for s in S],
            [v.data_ptr() for v in VH], nmax, chi.data_ptr(), w.data_ptr(), st.data_ptr())
    stream = torch.cuda.current_stream().cuda_stream
    if noalloc:
        _lib.check(_lib.rrsvd_truncate_noalloc(*args, stream))
    else:
        need = _lib.tebd_workspace_size(prm, m=m, n=n)
        buf, ptr = api.workspace(need, dev)
        _lib.check(_lib.rrsvd_truncate(*args, ptr, need, stream))
    torch.cuda.synchronize()
    return ([u.cpu().numpy() for u in U], [s.cpu().numpy() for s in S],
            [v.cpu().numpy()[:, :ni] for v, ni in zip(VH, n)], chi.cpu().numpy(), w.cpu().numpy(),
            st.cpu().numpy())


def _same(ref, got):
    U0, S0, V0, c0, w0, s0 = ref
    U1, S1, V1, c1, w1, s1 = got
    assert np.array_equal(c0, c1)
    assert np.array_equal(s0, s1)
    assert np.array_equal(w0, w1)
    for b in range(len(c0)):
        c = int(c0[b])
        scale = max(float(S0[b][0]), 1e-300)
        assert np.max(np.abs(S0[b] - S1[b])) <= 1e-10 * scale
        r0 = (U0[b][:, :c] * S0[b][None, :c]) @ V0[b][:c]
        r1 = (U1[b][:, :c] * S1[b][None, :c]) @ V1[b][:c]
        assert np.max(np.abs(r0 - r1)) <= 1e-10 * scale
        assert np.all(U1[b][:, c:] == 0) and np.all(S1[b][c:] == 0) and np.all(V1[b][c:] == 0)


def test_noalloc_matches_workspace_entry_point_twice():
    from paper_1504_00992_amd import _lib
    _lib.load()
    # call 1: 70 problems (two descriptor launches), ragged shapes, every
    # register QR class; call 2: a smaller batch of other shapes
    shapes1 = [(37, 53), (190, 140), (64, 90), (300, 200), (1, 10), (10, 1), (128, 128)] * 10
    shapes2 = [(90, 64), (200, 130)]
    for shapes, chi_max, sid in ((shapes1, 24, 3), (shapes2, 16, 4)):
        mats = _mats(shapes, 11 + sid)
        ref = _run(mats, chi_max, 10, 2, 1e-10, False, sid)
        got = _run(mats, chi_max, 10, 2, 1e-10, True, sid)
        _same(ref, got)
