"""Gradients of TEBD observables with respect to the gates and couplings.

Reverse mode over a TEBD run on the device, with checkpointed recomputation:
the forward keeps the state every K steps; the backward replays one segment
of K steps at a time with ``tebd_sweep_record`` (a copy of the state before
every sweep plus the sweep's tape), then undoes its sweeps in reverse order
with ``tebd_sweep_adjoint``.  Memory: one state per checkpoint plus, for the
segment being undone, 3 K states and 3 K tapes.

All arithmetic of the bond updates and their adjoints runs in the library's
kernels; this module moves buffers, keeps the sweep order (Sec. II.C, Eq.
defst3rd) and the random stream ids, and turns gate cotangents into coupling
derivatives on the host (the Frechet derivative of exp(-i tau h_b)).

Cotangent convention (also torch's): for a real loss L and complex z,
zbar = dL/dRe z + i dL/dIm z.
"""
import numpy as np
import torch

from . import _lib
from .api import BondWorkspace, _stream, workspace


def _snapshot(mps):
    return (mps.gamma.clone(), mps.lam.clone(), mps.chi.clone())


def _restore(mps, snap):
    mps.gamma.copy_(snap[0])
    mps.lam.copy_(snap[1])
    mps.chi.copy_(snap[2])


def _struct_of(mps, snap):
    return _lib.TebdMps(mps.n_chains, mps.n_sites, mps.d_max, mps.chi_max, mps.d.data_ptr(),
                        snap[0].data_ptr(), snap[1].data_ptr(), snap[2].data_ptr())


class CheckpointedTEBD:
    """Symmetric Trotter evolution of a DeviceMPS with a reverse pass.

    gates_half / gates_full: device [N-1, d_max^2, d_max^2] (complex128),
    shared by every chain, applied to the even bonds with tau = dt/2 and to
    the odd bonds with tau = dt.  Sweep s of the run uses stream_id = s, as
    ``api.TEBD`` does, so replays draw the same test matrices.
    """

    SWEEPS = ((0, "half"), (1, "full"), (0, "half"))

    def __init__(self, mps, gates_half, gates_full, chi_max, p=10, q=2, trunc_eps=1e-10,
                 seed=1504, lambda_floor=1e-14, precision=0, adaptive=2, checkpoint=10):
        if checkpoint < 1:
            raise ValueError("checkpoint must be >= 1")
        self.mps = mps
        self.gates = {"half": gates_half.contiguous(), "full": gates_full.contiguous()}
        self.prm = _lib.params(chi_max, p, q, trunc_eps, lambda_floor, seed, 0, precision,
                               adaptive)
        self.ws = BondWorkspace(mps, self.prm, adjoint=True)
        self.tape_bytes = _lib.tebd_tape_size(mps.struct(), self.prm)
        self.checkpoint = int(checkpoint)
        self.ckpts = {}
        self.steps = 0
        self._tapes = []

    # -- forward ------------------------------------------------------------
    def _sweep(self, parity, which, sweep_id, tape=None):
        self.prm.stream_id = sweep_id & 0xFFFFFFFF
        st = self.mps.struct()
        g = self.gates[which]
        if tape is None:
            _lib.check(_lib.tebd_sweep(st, g.data_ptr(), 0, parity, self.prm,
                                       self.ws.disc.data_ptr(), self.ws.status.data_ptr(),
                                       self.ws.ptr, self.ws.nbytes, _stream()))
        else:
            _lib.check(_lib.tebd_sweep_record(st, g.data_ptr(), 0, parity, self.prm,
                                              self.ws.disc.data_ptr(), self.ws.status.data_ptr(),
                                              tape[1], self.tape_bytes, self.ws.ptr,
                                              self.ws.nbytes, _stream()))

    def _step(self, step, tapes=None, snaps=None):
        for j, (parity, which) in enumerate(self.SWEEPS):
            tape = None
            if tapes is not None:
                snaps.append(_snapshot(self.mps))
                tape = tapes[len(snaps) - 1]
            self._sweep(parity, which, 3 * step + j, tape)

    def forward(self, steps):
        """Run `steps` time steps from the current state, keeping checkpoints."""
        self.ckpts = {}
        self.steps = int(steps)
        for s in range(self.steps):
            if s % self.checkpoint == 0:
                self.ckpts[s] = _snapshot(self.mps)
            self._step(s)

    # -- reverse ------------------------------------------------------------
    def _tape_pool(self, count):
        while len(self._tapes) < count:
            self._tapes.append(workspace(self.tape_bytes, self.mps.gamma.device))
        return self._tapes

    def backward(self, gamma_bar, lam_bar):
        """Cotangents of the final state -> those of the gates (and state).

        gamma_bar, lam_bar: device tensors shaped like mps.gamma / mps.lam
        (None means zero).  Returns (gate_bar_half, gate_bar_full,
        gamma_bar, lam_bar), the last two for the initial state.  The MPS is
        left in its final state.  Per-bond flags of the reverse sweeps are
        OR-ed into ``self.status`` (TEBD_DEV_BAD_STATE marks a skipped bond).
        """
        mps = self.mps
        final = _snapshot(mps)
        gb = torch.zeros_like(mps.gamma) if gamma_bar is None else gamma_bar.clone().contiguous()
        lb = torch.zeros_like(mps.lam) if lam_bar is None else lam_bar.clone().contiguous()
        gbar = {k: torch.zeros_like(v) for k, v in self.gates.items()}
        status = torch.zeros_like(self.ws.status)
        self.status = torch.zeros_like(self.ws.status)
        starts = sorted(self.ckpts)
        for si in reversed(range(len(starts))):
            s0 = starts[si]
            s1 = starts[si + 1] if si + 1 < len(starts) else self.steps
            _restore(mps, self.ckpts[s0])
            tapes = self._tape_pool(3 * (s1 - s0))
            snaps = []
            for s in range(s0, s1):
                self._step(s, tapes, snaps)
            for i in reversed(range(len(snaps))):
                parity, which = self.SWEEPS[i % 3]
                st_in = _struct_of(mps, snaps[i])
                _lib.check(_lib.tebd_sweep_adjoint(
                    st_in, self.gates[which].data_ptr(), 0, parity, self.prm, tapes[i][1],
                    self.tape_bytes, gb.data_ptr(), lb.data_ptr(), gbar[which].data_ptr(),
                    status.data_ptr(), self.ws.ptr, self.ws.nbytes, _stream()))
                self.status |= status
        _restore(mps, final)
        return gbar["half"], gbar["full"], gb, lb


class _Evolve(torch.autograd.Function):
    """Final (gamma, lambda) of a checkpointed run as a function of the gates."""

    @staticmethod
    def forward(ctx, gates_half, gates_full, driver, steps):
        driver.gates["half"].copy_(gates_half.detach())
        driver.gates["full"].copy_(gates_full.detach())
        driver.forward(steps)
        ctx.driver = driver
        return driver.mps.gamma.clone(), driver.mps.lam.clone()

    @staticmethod
    def backward(ctx, gamma_bar, lam_bar):
        gh, gf, _, _ = ctx.driver.backward(gamma_bar, lam_bar)
        return gh, gf, None, None


def evolve(gates_half, gates_full, driver, steps):
    """Differentiable TEBD run: returns the final (gamma, lambda) tensors.

    Backward runs the checkpointed adjoint of ``driver`` and returns the
    cotangents of the two gate stacks (torch's complex convention).
    """
    return _Evolve.apply(gates_half, gates_full, driver, steps)


def expectation(gamma, lam, op, site):
    """<O_site> of one chain by exact transfer-matrix contraction (torch ops).

    gamma [N, d_max, cap, cap], lam [N-1, cap] as stored by DeviceMPS; op is
    d_max x d_max (zero-padded).  Differentiable; used as a loss.
    """
    n = gamma.shape[0]
    cap = gamma.shape[-1]
    dmax = gamma.shape[1]
    op = torch.as_tensor(op, dtype=torch.complex128, device=gamma.device)
    eye = torch.eye(dmax, dtype=torch.complex128, device=gamma.device)
    env_o = torch.zeros((cap, cap), dtype=torch.complex128, device=gamma.device)
    env_o[0, 0] = 1.0
    env_n = env_o.clone()
    for k in range(n):
        a = gamma[k] * lam[k].to(torch.complex128)[None, None, :] if k < n - 1 else gamma[k]
        opk = op if k == site else eye
        env_o = torch.einsum("ab,iac,ij,jbd->cd", env_o, a.conj(), opk, a)
        env_n = torch.einsum("ab,iac,ibd->cd", env_n, a.conj(), a)
    return (env_o[0, 0] / env_n[0, 0]).real


def propagator_derivative(h, tau, dh):
    """d/dt exp(-i tau (h + t dh)) at t = 0 for Hermitian h and dh.

    Daleckii-Krein: with h = V diag(e) V^H, the derivative is
    V [(V^H (-i tau dh) V) o Phi] V^H, Phi_ij the divided difference of exp
    at x = -i tau e, written as exp(-i tau (e_i + e_j)/2) sinc(tau (e_i - e_j)/2)
    (exact, and stable for close eigenvalues).
    """
    h = np.asarray(h, dtype=np.complex128)
    e, v = np.linalg.eigh(0.5 * (h + h.conj().T))
    half = 0.5 * tau * (e[:, None] - e[None, :])
    phi = np.exp(-0.5j * tau * (e[:, None] + e[None, :])) * np.sinc(half / np.pi)
    inner = v.conj().T @ (-1j * tau * np.asarray(dh, dtype=np.complex128)) @ v
    return v @ (inner * phi) @ v.conj().T


def coupling_gradient(gate_bar, h, tau, dh):
    """dL/dtheta = Re tr(Gbar^H dG/dtheta) for G = exp(-i tau h(theta)).

    gate_bar: the bond's gate cotangent (at least k x k, k = dim of h).
    """
    k = np.asarray(h).shape[0]
    gb = np.asarray(gate_bar)[:k, :k]
    return float(np.real(np.sum(gb.conj() * propagator_derivative(h, tau, dh))))
