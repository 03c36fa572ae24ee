"""torch-facing wrappers of the C interface: memory, streams and bookkeeping.

torch supplies device memory and the current HIP stream; every step of the
bond update (Theta build, gate, sketch, QR, small SVD, truncation,
reabsorption) runs in the library's kernels.  Nothing here falls back to the
CPU: a missing library or device raises.
"""
import numpy as np
import torch

from . import _lib
from . import models


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _require_cuda(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")


def workspace(nbytes, device="cuda"):
    """A 256-byte aligned device buffer of at least nbytes."""
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off


def rrsvd_truncate(mats, chi_max, p=10, q=2, trunc_eps=1e-10, seed=1504, stream_id=0,
                   omegas=None, precision=0, ws=None):
    """Batched RRSVD truncation of a list of complex128 device matrices.

    Returns (U list [m x chi_max], S list [chi_max], VH list [chi_max x n],
    chi' int32 [batch], w float64 [batch], status int32 [batch]); entries past
    chi' are zero.  All outputs are device tensors, valid after the stream
    synchronises.
    """
    if not mats:
        raise ValueError("empty batch")
    for i, a in enumerate(mats):
        _require_cuda(a, f"mats[{i}]")
        if a.dtype != torch.complex128 or a.dim() != 2 or a.stride(1) != 1:
            raise ValueError(f"mats[{i}] must be a 2-D complex128 tensor with unit column stride")
    dev = mats[0].device
    prm = _lib.params(chi_max, p, q, trunc_eps, 1e-14, seed, stream_id, precision)
    m = [a.shape[0] for a in mats]
    n = [a.shape[1] for a in mats]
    nmax = max(n)
    U = [torch.zeros((mi, chi_max), dtype=torch.complex128, device=dev) for mi in m]
    S = [torch.zeros(chi_max, dtype=torch.float64, device=dev) for _ in mats]
    VH = [torch.zeros((chi_max, nmax), dtype=torch.complex128, device=dev) for _ in mats]
    chi = torch.zeros(len(mats), dtype=torch.int32, device=dev)
    w = torch.zeros(len(mats), dtype=torch.float64, device=dev)
    st = torch.zeros(len(mats), dtype=torch.int32, device=dev)
    need = _lib.tebd_workspace_size(prm, m=m, n=n)
    if ws is None or ws[0].numel() - 256 < need:
        ws = workspace(need, dev)
    om_ptrs = None
    if omegas is not None:
        om_ptrs = []
        for i, o in enumerate(omegas):
            _require_cuda(o, f"omegas[{i}]")
            if not o.is_contiguous() or o.dtype != torch.complex128:
                raise ValueError("omegas must be contiguous complex128")
            om_ptrs.append(o.data_ptr())
    _lib.check(_lib.rrsvd_truncate(m, n, [a.data_ptr() for a in mats], [a.stride(0) for a in mats],
                                   om_ptrs, prm, [u.data_ptr() for u in U], chi_max,
                                   [s.data_ptr() for s in S], [v.data_ptr() for v in VH], nmax,
                                   chi.data_ptr(), w.data_ptr(), st.data_ptr(), ws[1], need,
                                   _stream()))
    VH = [v[:, :ni] for v, ni in zip(VH, n)]
    return U, S, VH, chi, w, st


class DeviceMPS:
    """A batch of chains in Vidal form in fixed-capacity device arrays.

    gamma [n_chains, N, d_max, chi_max, chi_max] complex128,
    lam   [n_chains, N-1, chi_max] float64, chi [n_chains, N+1] int32,
    d [N] int32 -- the layout of tebd_mps in include/tebd_rrsvd.h.
    """

    def __init__(self, n_chains, dims, chi_max, device="cuda"):
        self.n_chains = int(n_chains)
        self.dims = [int(x) for x in dims]
        self.n_sites = len(dims)
        self.d_max = max(self.dims)
        self.chi_max = int(chi_max)
        N = self.n_sites
        self.gamma = torch.zeros((n_chains, N, self.d_max, chi_max, chi_max), dtype=torch.complex128,
                                 device=device)
        self.lam = torch.zeros((n_chains, N - 1, chi_max), dtype=torch.float64, device=device)
        self.chi = torch.ones((n_chains, N + 1), dtype=torch.int32, device=device)
        self.d = torch.tensor(self.dims, dtype=torch.int32, device=device)

    @classmethod
    def product_state(cls, n_chains, dims, levels, chi_max, device="cuda"):
        mps = cls(n_chains, dims, chi_max, device)
        g = torch.zeros_like(mps.gamma[0])
        for k, lv in enumerate(levels):
            g[k, lv, 0, 0] = 1.0
        mps.gamma[:] = g
        mps.lam[:, :, 0] = 1.0
        return mps

    @classmethod
    def from_host(cls, chains, dims, chi_max, device="cuda"):
        """chains: list of (gammas, lambdas); gammas[k] shape (d_k, chi_k, chi_k+1)."""
        mps = cls(len(chains), dims, chi_max, device)
        g = np.zeros(tuple(mps.gamma.shape), dtype=np.complex128)
        lam = np.zeros(tuple(mps.lam.shape), dtype=np.float64)
        chi = np.ones(tuple(mps.chi.shape), dtype=np.int32)
        for c, (gammas, lambdas) in enumerate(chains):
            for k, gk in enumerate(gammas):
                d, cl, cr = gk.shape
                if cl > chi_max or cr > chi_max:
                    raise ValueError("bond dimension exceeds chi_max")
                g[c, k, :d, :cl, :cr] = gk
                chi[c, k] = cl
                chi[c, k + 1] = cr
            for b, lb in enumerate(lambdas):
                lam[c, b, :len(lb)] = lb
        mps.gamma.copy_(torch.from_numpy(g))
        mps.lam.copy_(torch.from_numpy(lam))
        mps.chi.copy_(torch.from_numpy(chi))
        return mps

    def to_host(self, chain=0):
        """(gammas, lambdas) of one chain trimmed to its current bond dims."""
        g = self.gamma[chain].cpu().numpy()
        lam = self.lam[chain].cpu().numpy()
        chi = self.chi[chain].cpu().numpy()
        gammas = [g[k, :self.dims[k], :chi[k], :chi[k + 1]].copy() for k in range(self.n_sites)]
        lambdas = [lam[b, :chi[b + 1]].copy() for b in range(self.n_sites - 1)]
        return gammas, lambdas

    def struct(self):
        return _lib.TebdMps(self.n_chains, self.n_sites, self.d_max, self.chi_max,
                            self.d.data_ptr(), self.gamma.data_ptr(), self.lam.data_ptr(),
                            self.chi.data_ptr())


class BondWorkspace:
    """Workspace and per-bond outputs sized for sweeps over one DeviceMPS
    (adjoint=True: also for the reverse sweeps)."""

    def __init__(self, mps, prm, adjoint=False):
        if adjoint:
            self.nbytes = _lib.tebd_adjoint_workspace_size(mps.struct(), prm)
        else:
            self.nbytes = _lib.tebd_workspace_size(prm, mps=mps.struct())
        self.buf, self.ptr = workspace(self.nbytes, mps.gamma.device)
        dev = mps.gamma.device
        self.disc = torch.zeros((mps.n_chains, mps.n_sites - 1), dtype=torch.float64, device=dev)
        self.status = torch.zeros((mps.n_chains, mps.n_sites - 1), dtype=torch.int32, device=dev)


def tebd_sweep(mps, gates, parity, prm, ws, gate_chain_stride=0):
    """One parity sweep over every chain (gates: device [.., N-1, d^2, d^2])."""
    _require_cuda(gates, "gates")
    st = mps.struct()
    _lib.check(_lib.tebd_sweep(st, gates.data_ptr(), gate_chain_stride, parity, prm,
                               ws.disc.data_ptr(), ws.status.data_ptr(), ws.ptr, ws.nbytes,
                               _stream()))


def tebd_bond_update(mps, chain, bond, gate, prm, ws, disc=None, status=None):
    """Update one bond of one chain; gate is a device (d_max^2 x d_max^2) block."""
    _require_cuda(gate, "gate")
    st = mps.struct()
    disc = ws.disc[chain, bond:] if disc is None else disc
    status = ws.status[chain, bond:] if status is None else status
    _lib.check(_lib.tebd_bond_update(st, chain, bond, gate.data_ptr(), prm, disc.data_ptr(),
                                     status.data_ptr(), ws.ptr, ws.nbytes, _stream()))


def trotter_schedule(order=2):
    """(parity, tau / dt) of the sweeps of one time step.

    order 2: the symmetric splitting of Sec. II.C, Eq. (defst3rd): even
    bonds for dt/2, odd bonds for dt, even bonds for dt/2.  order 4: one of
    the higher-order schemes Sec. II.C refers to, Suzuki's fourth-order
    fractal product of five symmetric steps of lengths w dt, w dt,
    (1 - 4w) dt, w dt, w dt with w = 1 / (4 - 4^(1/3)) (local error
    O(dt^5)); 15 sweeps, the meeting half sweeps not merged."""
    if order == 2:
        return ((0, 0.5), (1, 1.0), (0, 0.5))
    if order == 4:
        w = 1.0 / (4.0 - 4.0 ** (1.0 / 3.0))
        sched = []
        for x in (w, w, 1.0 - 4.0 * w, w, w):
            sched += [(0, 0.5 * x), (1, x), (0, 0.5 * x)]
        return tuple(sched)
    raise ValueError("order must be 2 or 4")


class TEBD:
    """Trotter time stepping (Sec. II.C) on a DeviceMPS.

    order 2: one step = three sweeps (Eq. defst3rd): even bonds with
    tau = dt/2, odd bonds with dt, even bonds with dt/2.  order 4: fifteen
    sweeps (trotter_schedule).  Sweep s of the run draws its Gaussian test
    matrices with stream_id = s, so every bond update has its own Omega.
    """

    def __init__(self, mps, bond_hams, dt, chi_max, p=10, q=2, trunc_eps=1e-10, seed=1504,
                 lambda_floor=1e-14, precision=0, adaptive=0, order=2, generators=None):
        """bond_hams: two-site Hamiltonians (gates exp(-i tau h_b)); or, for a
        density matrix held as an MPO over the operator space (Sec. II, mixed
        states; models.liouville_generators), generators: the bond
        generators L_b (gates exp(tau L_b)) and bond_hams unused."""
        self.mps = mps
        self.dt = dt
        dev = mps.gamma.device
        self.schedule = []
        stacks = {}
        for parity, frac in trotter_schedule(order):
            if frac not in stacks:
                if generators is not None:
                    g = models.generator_gate_stack(mps.dims, generators, frac * dt)
                else:
                    g = models.gate_stack(mps.dims, bond_hams, frac * dt)
                stacks[frac] = torch.from_numpy(g).to(dev)
            self.schedule.append((parity, stacks[frac]))
        self.g_half = stacks[0.5] if 0.5 in stacks else None
        self.g_full = stacks[1.0] if 1.0 in stacks else None
        self.prm = _lib.params(chi_max, p, q, trunc_eps, lambda_floor, seed, 0, precision, adaptive)
        self.ws = BondWorkspace(mps, self.prm)
        self.sweeps_done = 0
        self.history = []

    def sweep(self, parity, gates, record=False):
        self.prm.stream_id = self.sweeps_done & 0xFFFFFFFF
        tebd_sweep(self.mps, gates, parity, self.prm, self.ws)
        self.sweeps_done += 1
        if record:
            self.history.append((parity, self.ws.disc.clone(), self.ws.status.clone()))

    def step(self, record=False):
        for parity, gates in self.schedule:
            self.sweep(parity, gates, record)

    def bond_updates_per_step(self):
        n = self.mps.n_sites
        return self.mps.n_chains * (n - 1)


class GraphTEBD:
    """Trotter steps of a TEBD driver captured in HIP graphs and replayed.

    The driver must use a rank mode that never waits for the host (adaptive
    0 or 1: the second pass of the two-stage rank is skipped on the device),
    so that every launch of a sweep can be captured.  `steps` steps are
    captured in graphs of at most `steps_per_graph` steps each; each sweep's
    Gaussian test matrices follow its position in the run (as in eager
    stepping from sweeps_done = 0), so a replay from a given state computes
    exactly what eager stepping from that state does.  Capturing does not
    run anything: the MPS is left as it was.  replay() runs all graphs in
    order on the current stream.
    """

    def __init__(self, drv, steps, steps_per_graph=25):
        if drv.prm.adaptive not in (0, 1):
            raise ValueError("graph capture needs adaptive = 0 or 1 (no host round trip)")
        mps = drv.mps
        snap = (mps.gamma.clone(), mps.lam.clone(), mps.chi.clone())
        # one eager step first: the library creates its side streams and sets
        # kernel attributes on first use, which capture does not allow
        drv.sweeps_done = 0
        drv.step()
        torch.cuda.synchronize()
        self._restore(mps, snap)
        drv.sweeps_done = 0
        self.drv = drv
        self.steps = int(steps)
        self.graphs = []
        stream = torch.cuda.Stream()
        done = 0
        while done < self.steps:
            k = min(int(steps_per_graph), self.steps - done)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                for _ in range(k):
                    drv.step()
            self.graphs.append(g)
            done += k
        torch.cuda.synchronize()
        drv.sweeps_done = 0

    @staticmethod
    def _restore(mps, snap):
        mps.gamma.copy_(snap[0])
        mps.lam.copy_(snap[1])
        mps.chi.copy_(snap[2])

    def replay(self):
        for g in self.graphs:
            g.replay()
