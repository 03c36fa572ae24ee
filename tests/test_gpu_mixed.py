"""Mixed-precision path (complex FP32 sketch and power-iteration products,
FP64 QR, projection, small SVD and reabsorption) against the FP64 oracle.

Tolerance 1e-5 (normwise for singular values, absolute for observables):
the FP32 products perturb the sketched subspace at the 1e-7 level, and the
FP64 projection turns that into much smaller Ritz-value errors; 1e-5 is the
bound stated for this path.  The measured errors are printed.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import models as om
from oracle import mps as omps
from oracle import philox, rrsvd as orr

pytestmark = pytest.mark.gpu
SEED = 1504


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


@pytest.mark.parametrize("m,n,chi_max", [(300, 300, 50), (700, 650, 64), (1280, 1280, 128)])
def test_mixed_rrsvd_against_fp64_oracle(m, n, chi_max):
    from paper_1504_00992_amd import api
    gen = wl.rng(m + 7 * n)
    s = np.exp(-np.arange(min(m, n)) / (chi_max / 8.0))
    a = wl.known_spectrum(m, n, s, gen)
    U, S, VH, chi, w, st = api.rrsvd_truncate([torch.from_numpy(a).cuda()], chi_max, 10, 2, 1e-10,
                                              SEED, 0, precision=1)
    torch.cuda.synchronize()
    l = orr.sketch_width(chi_max, 10, m, n)
    ou, os_, ovh, ochi, ow, ost = orr.truncate_rrsvd(a, philox.gaussian_omega(n, l, SEED, 0, 0), 2,
                                                     chi_max, 1e-10)
    c = int(chi[0].item())
    assert c == ochi
    sv = S[0].cpu().numpy()[:c]
    err = np.max(np.abs(sv - os_)) / os_[0]
    print(f"mixed rrsvd {m}x{n}: max |ds|/s1 = {err:.2e}")
    assert err < 1e-5
    assert abs(w[0].item() - ow) < 1e-6
    rec = (U[0].cpu().numpy()[:, :c] * sv[None, :]) @ VH[0].cpu().numpy()[:c]
    assert np.max(np.abs(rec - (ou * os_[None, :]) @ ovh)) < 1e-5 * os_[0]


def test_mixed_tebd_spin_boson_against_fp64_oracle():
    from paper_1504_00992_amd import api
    n, d, dt, steps, chi_max = 8, 6, 0.05, 8, 24
    dims, hb = om.spin_boson_chain(n, d, 1.0, 0.5, 1.0, 0.5)
    dev = api.DeviceMPS.product_state(1, dims, [0] * n, chi_max)
    drv = api.TEBD(dev, hb, dt, chi_max, p=10, q=2, trunc_eps=1e-10, seed=SEED, precision=1)
    for _ in range(steps):
        drv.step()
    torch.cuda.synchronize()
    cache = {}

    def gfn(b, tau):
        if (b, tau) not in cache:
            cache[(b, tau)] = om.gate(hb[b], tau)
        return cache[(b, tau)]
    ref = omps.TEBD(omps.basis_product_state(dims, [0] * n), gfn, dt, chi_max, 1e-10,
                    method="rrsvd", p=10, q=2, seed=SEED)
    for _ in range(steps):
        ref.step()
    gam, lam = dev.to_host(0)
    gm = omps.MPS(gam, lam)
    num = np.diag(np.arange(d)).astype(np.complex128)
    errs = [abs(omps.expectation(gm, om.Z, 0).real - omps.expectation(ref.mps, om.Z, 0).real)]
    for i in range(1, n):
        errs.append(abs(omps.expectation(gm, num, i).real - omps.expectation(ref.mps, num, i).real))
    print(f"mixed TEBD: max observable error {max(errs):.2e}")
    assert max(errs) < 1e-5
    assert abs(omps.norm2(gm) - 1.0) < 1e-8


def test_mixed_spin_boson_chi128_full_run_against_fp64_oracle():
    # The mixed-precision workload at full size: 16 spin-boson chains, N = 100,
    # d = 10, chi_max = 128, 200 steps, adaptive rank, FP32 sketch and
    # power-iteration products.  Chain 0 against the FP64 oracle run with the
    # same test matrices (tests/golden/spin_boson_n100_chi128.txt): bond
    # dimensions exactly, lambda and <sigma_z> within the 1e-5 bound of this
    # path.
    import os
    from paper_1504_00992_amd import api, models as pm
    path = os.path.join(os.path.dirname(__file__), "golden", "spin_boson_n100_chi128.txt")
    z, lams = {}, {}
    for line in open(path):
        t = line.split()
        if not t or t[0].startswith("#"):
            continue
        if t[0] == "obs":
            z[int(t[1])] = float(t[2])
        elif t[0] == "lam":
            lams[int(t[1])] = np.array([float(x) for x in t[2:]])
    n, d = 100, 10
    dims, hb = pm.spin_boson(n, d, 1.0, 0.5, 1.0, 0.5)
    dev = api.DeviceMPS.product_state(16, dims, [0] * n, 128)
    drv = api.TEBD(dev, hb, 0.05, 128, p=10, q=2, trunc_eps=1e-10, seed=SEED, adaptive=2,
                   precision=1)
    zerr = 0.0
    for s in range(1, 201):
        drv.step()
        if s in z:
            torch.cuda.synchronize()
            gam, lam = dev.to_host(0)
            zerr = max(zerr, abs(omps.expectation(omps.MPS(gam, lam), om.Z, 0).real - z[s]))
    gam, lam = dev.to_host(0)
    assert [len(x) for x in lam] == [len(lams[b]) for b in range(n - 1)]
    lerr = max(float(np.max(np.abs(lam[b] - lams[b]))) for b in range(n - 1))
    print(f"mixed chi_max=128 spin-boson: max |d lambda| {lerr:.2e}, max |d <sigma_z>| {zerr:.2e}")
    assert lerr < 1e-5 and zerr < 1e-5
