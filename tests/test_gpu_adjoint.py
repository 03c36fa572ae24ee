"""GPU parity of the reverse mode (tebd_sweep_record / tebd_sweep_adjoint).

* One sweep: the cotangents of every Gamma and lambda and of every gate,
  for random states and gates, against the oracle's ``bond_adjoint``
  applied to the oracle's own step-by-step RRSVD of the same bonds (same
  Philox test matrices): element by element, 1e-9 relative to the largest
  entry of each array; padding exactly zero.  The output cotangents come
  from a loss that does not depend on the phase of a singular pair,
  evaluated on each side's own result (the two sides may choose different
  phases; a real observable never sees them).
* Whole runs of the XX chain with random fields: d<Z_0(T)>/dJ_b against the
  oracle's reverse mode over the same algorithm (1e-9), and, at N = 40 with
  50 steps, against the stored references of tests/golden (reverse mode
  over the exact-SVD run, central differences, free fermions).
* Checkpointing changes nothing (bitwise), the torch.autograd path agrees
  with the host Frechet route, and a tape that does not describe the state
  is refused per bond.
"""
import os

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import adjoint as oa
from oracle import models as om
from oracle import mps as omps
from oracle import philox

pytestmark = pytest.mark.gpu
SEED = 1504
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"


def _gate_stack(dims, gen):
    dmax = max(dims)
    gates = []
    stack = np.zeros((len(dims) - 1, dmax * dmax, dmax * dmax), dtype=np.complex128)
    for b in range(len(dims) - 1):
        k = dims[b] * dims[b + 1]
        g = wl.random_unitary(k, gen)
        gates.append(g)
        stack[b, :k, :k] = g
    return gates, stack


def _loss_weights(dims, chis, gen):
    """Random weights of a loss that does not depend on the phase of any
    singular pair: sum_k W_k o |Gamma_k|^2 + sum_b w_b . lambda_b
    + sum_b Re <V_b, Theta_b> with Theta_b the two-site block of bond b, for
    the bonds of the sweep (their outer bonds keep their gauge)."""
    n = len(dims)
    w_gam = [gen.standard_normal((d, chis[k], chis[k + 1])) for k, d in enumerate(dims)]
    w_lam = [gen.standard_normal(chis[b + 1]) for b in range(n - 1)]
    w_th = [wl.ginibre(dims[b] * chis[b], dims[b + 1] * chis[b + 2], gen)
            for b in range(n - 1)]
    return w_gam, w_lam, w_th


def _loss_cotangents(gammas, lambdas, weights, parity):
    """Cotangents of that loss (torch CPU autograd) at the given state."""
    w_gam, w_lam, w_th = weights
    n = len(gammas)
    gs = [torch.tensor(np.array(g), requires_grad=True) for g in gammas]
    ls = [torch.tensor(np.array(l), requires_grad=True) for l in lambdas]
    one = torch.ones(1, dtype=torch.float64)
    loss = torch.zeros((), dtype=torch.float64)
    for k in range(n):
        loss = loss + (torch.from_numpy(w_gam[k]) * gs[k].abs() ** 2).sum()
    for b in range(n - 1):
        loss = loss + (torch.from_numpy(w_lam[b]) * ls[b]).sum()
        if b % 2 != parity:
            continue
        ll = ls[b - 1] if b >= 1 else one
        lr = ls[b + 1] if b + 1 <= n - 2 else one
        th = torch.einsum("a,iag,g,jgc,c->iajc", ll.to(torch.complex128), gs[b],
                          ls[b].to(torch.complex128), gs[b + 1], lr.to(torch.complex128))
        th = th.reshape(w_th[b].shape)
        loss = loss + (torch.from_numpy(w_th[b]).conj() * th).real.sum()
    loss.backward()
    return [g.grad.numpy().copy() for g in gs], [l.grad.numpy().copy() for l in ls]


def _rel(a, b):
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)


@pytest.mark.parametrize("dims,chis,parity,chi_max,p,adaptive", [
    ([2, 3, 2, 3, 2, 2], [1, 2, 4, 5, 4, 2, 1], 0, 6, 4, 0),
    ([2, 3, 2, 3, 2, 2], [1, 2, 4, 5, 4, 2, 1], 1, 6, 4, 0),
    ([2, 2, 2, 2, 2], [1, 2, 4, 4, 2, 1], 0, 8, 10, 1),
    ([3, 3, 3, 3], [1, 3, 7, 3, 1], 1, 5, 3, 0),
    ([2, 2, 2, 2, 2, 2, 2], [1, 2, 4, 6, 6, 4, 2, 1], 1, 12, 6, 1),
])
def test_sweep_adjoint_matches_oracle(dims, chis, parity, chi_max, p, adaptive):
    from paper_1504_00992_amd import _lib, api
    n = len(dims)
    gen = wl.rng(31 + 7 * parity + len(dims))
    gam, lam = wl.random_vidal_chain(dims, chis, gen)
    gates, stack = _gate_stack(dims, gen)
    cap = max(max(chis), chi_max)
    eps, sid = 1e-10, 7
    dev = api.DeviceMPS.from_host([(gam, lam)], dims, cap)
    before = (dev.gamma.clone(), dev.lam.clone(), dev.chi.clone())
    prm = _lib.params(chi_max, p, 2, eps, 1e-14, SEED, sid, 0, adaptive)
    ws = api.BondWorkspace(dev, prm, adjoint=True)
    tbytes = _lib.tebd_tape_size(dev.struct(), prm)
    tape = api.workspace(tbytes)
    gd = torch.from_numpy(stack).cuda()
    print(f"record dims={dims} chis={chis} parity={parity}", flush=True)
    _lib.check(_lib.tebd_sweep_record(dev.struct(), gd.data_ptr(), 0, parity, prm,
                                      ws.disc.data_ptr(), ws.status.data_ptr(), tape[1], tbytes,
                                      ws.ptr, ws.nbytes, api._stream()))
    torch.cuda.synchronize()
    after = dev.chi[0].cpu().numpy()
    # cotangents of a gauge-invariant loss of the state after the sweep,
    # evaluated on each side's own state
    g_gam, g_lam = dev.to_host(0)
    weights = _loss_weights(dims, after, gen)
    gbar_g, lbar_g = _loss_cotangents(g_gam, g_lam, weights, parity)
    cg = np.zeros(tuple(dev.gamma.shape), dtype=np.complex128)
    cl = np.zeros(tuple(dev.lam.shape), dtype=np.float64)
    for k, d in enumerate(dims):
        cg[0, k, :d, :after[k], :after[k + 1]] = gbar_g[k]
    for b in range(n - 1):
        cl[0, b, :after[b + 1]] = lbar_g[b]
    gbar = torch.from_numpy(cg).cuda()
    lbar = torch.from_numpy(cl).cuda()
    gate_bar = torch.zeros_like(gd)
    status = torch.full_like(ws.status, -1)
    st_in = _lib.TebdMps(1, n, max(dims), cap, dev.d.data_ptr(), before[0].data_ptr(),
                         before[1].data_ptr(), before[2].data_ptr())
    print("adjoint", flush=True)
    _lib.check(_lib.tebd_sweep_adjoint(st_in, gd.data_ptr(), 0, parity, prm, tape[1], tbytes,
                                       gbar.data_ptr(), lbar.data_ptr(), gate_bar.data_ptr(),
                                       status.data_ptr(), ws.ptr, ws.nbytes, api._stream()))
    torch.cuda.synchronize()
    # oracle: the same bond updates, then bond_adjoint on each
    ref = omps.MPS(gam, lam)
    method = "rrsvd_adaptive" if adaptive else "rrsvd"
    recs = []
    for b in range(parity, n - 1, 2):
        ncol = dims[b + 1] * ref.chis()[b + 2]

        def omega_of(l, ncol=ncol, b=b):
            return philox.gaussian_omega(ncol, l, SEED, b, sid)
        recs.append(oa.recorded_bond_update(ref, b, gates[b], chi_max, eps, method, omega_of, 2,
                                            p))
    assert ref.chis() == list(after)
    exp_g, exp_l = _loss_cotangents(ref.gammas, ref.lambdas, weights, parity)
    cot_g = [x.copy() for x in exp_g]
    cot_l = [x.copy() for x in exp_l]
    exp_gate = {}
    for rec in recs:
        b = rec["b"]
        assert rec["chi"] == after[b + 1], (b, rec["chi"], after[b + 1])
        out = oa.bond_adjoint(rec["gk"], rec["gk1"], rec["lam_l"], rec["lam_m"], rec["lam_r"],
                              rec["gate"], rec["u"], rec["s"], rec["vh"], rec["chi"],
                              exp_g[b], exp_g[b + 1], exp_l[b])
        exp_g[b], exp_g[b + 1], exp_l[b] = out["gk_bar"], out["gk1_bar"], out["lam_m_bar"]
        exp_gate[b] = out["gate_bar"]
    for rec in recs:  # contributions to the lambdas the sweep only read
        b = rec["b"]
        out = oa.bond_adjoint(rec["gk"], rec["gk1"], rec["lam_l"], rec["lam_m"], rec["lam_r"],
                              rec["gate"], rec["u"], rec["s"], rec["vh"], rec["chi"],
                              cot_g[b], cot_g[b + 1], cot_l[b])
        if b >= 1:
            exp_l[b - 1] = exp_l[b - 1] + out["lam_l_bar"]
        if b + 1 <= n - 2:
            exp_l[b + 1] = exp_l[b + 1] + out["lam_r_bar"]
    assert np.all(status.cpu().numpy()[0, parity::2] == 0)
    got_g = gbar.cpu().numpy()[0]
    got_l = lbar.cpu().numpy()[0]
    for k, d in enumerate(dims):
        blk = got_g[k, :d, :chis[k], :chis[k + 1]]
        assert blk.shape == exp_g[k].shape
        assert _rel(blk, exp_g[k]) < 1e-9, (k, _rel(blk, exp_g[k]))
        pad = got_g[k].copy()
        pad[:d, :chis[k], :chis[k + 1]] = 0
        assert np.all(pad == 0)
    for b in range(n - 1):
        assert _rel(got_l[b, :chis[b + 1]], exp_l[b]) < 1e-9, (b, got_l[b], exp_l[b])
        assert np.all(got_l[b, chis[b + 1]:] == 0)
    gb = gate_bar.cpu().numpy()
    for b in range(n - 1):
        k = dims[b] * dims[b + 1]
        if b in exp_gate:
            assert _rel(gb[b, :k, :k], exp_gate[b]) < 1e-9, b
        else:
            assert np.all(gb[b] == 0)


def test_adjoint_refuses_a_tape_of_another_sweep():
    from paper_1504_00992_amd import _lib, api
    dims, chis = [2, 2, 2, 2, 2], [1, 2, 4, 4, 2, 1]
    gen = wl.rng(5)
    gam, lam = wl.random_vidal_chain(dims, chis, gen)
    _, stack = _gate_stack(dims, gen)
    dev = api.DeviceMPS.from_host([(gam, lam)], dims, 8)
    before = (dev.gamma.clone(), dev.lam.clone(), dev.chi.clone())
    prm = _lib.params(8, 4, 2, 1e-10)
    ws = api.BondWorkspace(dev, prm, adjoint=True)
    tbytes = _lib.tebd_tape_size(dev.struct(), prm)
    tape = api.workspace(tbytes)
    gd = torch.from_numpy(stack).cuda()
    _lib.check(_lib.tebd_sweep_record(dev.struct(), gd.data_ptr(), 0, 0, prm, ws.disc.data_ptr(),
                                      ws.status.data_ptr(), tape[1], tbytes, ws.ptr, ws.nbytes,
                                      api._stream()))
    gbar = torch.ones_like(dev.gamma)
    lbar = torch.ones_like(dev.lam)
    gate_bar = torch.zeros_like(gd)
    status = torch.zeros_like(ws.status)
    st_in = _lib.TebdMps(1, 5, 2, 8, dev.d.data_ptr(), before[0].data_ptr(), before[1].data_ptr(),
                         before[2].data_ptr())
    # parity 1 with the tape of a parity-0 sweep: no slot matches its bond
    _lib.check(_lib.tebd_sweep_adjoint(st_in, gd.data_ptr(), 0, 1, prm, tape[1], tbytes,
                                       gbar.data_ptr(), lbar.data_ptr(), gate_bar.data_ptr(),
                                       status.data_ptr(), ws.ptr, ws.nbytes, api._stream()))
    torch.cuda.synchronize()
    st = status.cpu().numpy()[0]
    assert np.all(st[1::2] == _lib.DEV_BAD_STATE)
    assert torch.all(gbar == 1) and torch.all(lbar == 1) and torch.all(gate_bar == 0)


# ---------------------------------------------------------------------------
# Whole runs: XX chain with random fields, gradient of <Z_0(T)> w.r.t. J_b.

HOP = 0.5 * (np.kron(om.X, om.X) + np.kron(om.Y, om.Y))


def _gpu_gradient(n_sites, steps, dt, chi_max, eps, checkpoint, seed, adaptive=1, p=10, q=2,
                  return_driver=False):
    from paper_1504_00992_amd import api, gradient, models as pm
    J, h = wl.xx_couplings(n_sites, seed=SEED)
    dims, hb = pm.xx_chain(J, h)
    g_half = torch.from_numpy(pm.gate_stack(dims, hb, 0.5 * dt)).cuda()
    g_full = torch.from_numpy(pm.gate_stack(dims, hb, dt)).cuda()
    mps = api.DeviceMPS.product_state(1, dims, wl.neel_levels(n_sites), chi_max)
    drv = gradient.CheckpointedTEBD(mps, g_half, g_full, chi_max, p, q, eps, seed,
                                    adaptive=adaptive, checkpoint=checkpoint)
    drv.forward(steps)
    gam = mps.gamma[0].clone().requires_grad_(True)
    lam = mps.lam[0].clone().requires_grad_(True)
    val = gradient.expectation(gam, lam, om.Z, 0)
    val.backward()
    gb = torch.zeros_like(mps.gamma)
    lb = torch.zeros_like(mps.lam)
    gb[0] = gam.grad
    lb[0] = lam.grad
    gh, gf, _, _ = drv.backward(gb, lb)
    torch.cuda.synchronize()
    assert int(drv.status.max().item()) == 0
    gh, gf = gh.cpu().numpy(), gf.cpu().numpy()
    grad = np.array([gradient.coupling_gradient(gh[b], hb[b], 0.5 * dt, HOP)
                     + gradient.coupling_gradient(gf[b], hb[b], dt, HOP)
                     for b in range(n_sites - 1)])
    out = (float(val.item()), grad, gh, gf)
    return out + (drv,) if return_driver else out


def _oracle_gradient(n_sites, steps, dt, chi_max, eps, seed):
    J, h = wl.xx_couplings(n_sites, seed=SEED)
    dims, hb = om.xx_field(J, h)
    cache = {}

    def g(b, tau):
        if (b, tau) not in cache:
            cache[(b, tau)] = om.gate(hb[b], tau)
        return cache[(b, tau)]
    mps0 = omps.basis_product_state(dims, wl.neel_levels(n_sites))
    val, grad, _, _ = oa.tebd_gradient(mps0, g, lambda b: hb[b],
                                       lambda b, k: HOP if b == k else None, n_sites - 1, dt,
                                       steps, chi_max, eps, om.Z, 0, method="rrsvd_adaptive",
                                       seed=seed)
    return val, grad


def test_gradient_matches_oracle_reverse_mode_small():
    args = dict(n_sites=8, steps=12, dt=0.02, chi_max=16, eps=1e-10)
    print("gpu gradient N=8", flush=True)
    val, grad, _, _ = _gpu_gradient(**args, checkpoint=5, seed=77)
    v_ref, g_ref = _oracle_gradient(**args, seed=77)
    assert abs(val - v_ref) < 1e-10
    assert _rel(grad, g_ref) < 1e-9, (grad, g_ref)


def test_checkpoint_interval_does_not_change_the_gradient():
    args = dict(n_sites=8, steps=7, dt=0.05, chi_max=16, eps=1e-10, seed=3)
    runs = [_gpu_gradient(**args, checkpoint=k) for k in (1, 3, 7)]
    for _, grad, gh, gf in runs[1:]:
        assert np.array_equal(gh, runs[0][2]) and np.array_equal(gf, runs[0][3])
        assert np.array_equal(grad, runs[0][1])


def test_autograd_path_matches_frechet_route():
    from paper_1504_00992_amd import api, gradient, models as pm
    n_sites, steps, dt, chi_max = 6, 5, 0.05, 16
    J, h = wl.xx_couplings(n_sites, seed=SEED)
    dims, hb = pm.xx_chain(J, h)
    hop = torch.from_numpy(HOP).cuda()
    const = [torch.from_numpy(hb[b] - J[b] * HOP).cuda() for b in range(n_sites - 1)]
    jt = torch.tensor(J, dtype=torch.float64, device="cuda", requires_grad=True)

    def stack(tau):
        hs = torch.stack([jt[b].to(torch.complex128) * hop + const[b] for b in range(n_sites - 1)])
        return torch.linalg.matrix_exp(-1j * tau * hs)
    mps = api.DeviceMPS.product_state(1, dims, wl.neel_levels(n_sites), chi_max)
    drv = gradient.CheckpointedTEBD(mps, stack(0.5 * dt).detach(), stack(dt).detach(), chi_max,
                                    checkpoint=2, seed=11)
    gam, lam = gradient.evolve(stack(0.5 * dt), stack(dt), drv, steps)
    loss = gradient.expectation(gam[0], lam[0], om.Z, 0)
    loss.backward()
    auto = jt.grad.cpu().numpy()
    _, ref, _, _ = _gpu_gradient(n_sites, steps, dt, chi_max, 1e-10, 2, 11)
    assert _rel(auto, ref) < 1e-10, (auto, ref)


def _golden():
    path = os.path.join(HERE, "golden", "xx_n40_gradient.txt")
    meta = {}
    with open(path) as f:
        for line in f:
            if line.startswith("# value_") or line.startswith("# max_chi"):
                key, val = line[2:].split()
                meta[key] = float(val)
    return meta, np.loadtxt(path)


def test_gradient_n40_matches_references():
    meta, ref = _golden()
    print("gpu gradient N=40, 50 steps, checkpoint 10", flush=True)
    val, grad, _, _ = _gpu_gradient(40, 50, 0.02, 64, 1e-10, 10, SEED)
    assert abs(val - meta["value_tebd"]) < 1e-10
    scale = np.max(np.abs(ref[:, 3]))
    err_rev = np.max(np.abs(grad - ref[:, 2])) / scale
    err_fd = np.max(np.abs(grad - ref[:, 3])) / scale
    err_ff = np.max(np.abs(grad - ref[:, 4])) / scale
    print(f"relative to max|dL/dJ|: vs exact-SVD reverse {err_rev:.2e}, vs finite differences "
          f"{err_fd:.2e}, vs free fermions {err_ff:.2e}", flush=True)
    assert err_rev < 1e-8
    assert err_fd < 1e-7
    assert err_ff < 2e-5


def test_recording_does_not_change_the_sweep():
    from paper_1504_00992_amd import _lib, api
    dims, chis = [2, 3, 3, 3, 2], [1, 2, 6, 6, 2, 1]
    gen = wl.rng(17)
    gam, lam = wl.random_vidal_chain(dims, chis, gen)
    _, stack = _gate_stack(dims, gen)
    gd = torch.from_numpy(stack).cuda()
    prm = _lib.params(5, 3, 2, 1e-10, 1e-14, SEED, 3, 0, 1)
    a = api.DeviceMPS.from_host([(gam, lam)] * 2, dims, 8)
    b = api.DeviceMPS.from_host([(gam, lam)] * 2, dims, 8)
    wa = api.BondWorkspace(a, prm)
    wb = api.BondWorkspace(b, prm, adjoint=True)
    tbytes = _lib.tebd_tape_size(b.struct(), prm)
    tape = api.workspace(tbytes)
    for parity in (0, 1, 0):
        api.tebd_sweep(a, gd, parity, prm, wa)
        _lib.check(_lib.tebd_sweep_record(b.struct(), gd.data_ptr(), 0, parity, prm,
                                          wb.disc.data_ptr(), wb.status.data_ptr(), tape[1],
                                          tbytes, wb.ptr, wb.nbytes, api._stream()))
    torch.cuda.synchronize()
    assert torch.equal(a.gamma, b.gamma) and torch.equal(a.lam, b.lam)
    assert torch.equal(a.chi, b.chi) and torch.equal(wa.disc, wb.disc)
    assert torch.equal(wa.status, wb.status)
