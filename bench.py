"""Throughput of the batched TEBD bond update with RRSVD on one MI355X.

Workload (default): 16 independent chain-mapped spin-boson chains (Eq. H_1D:
spin-1/2 plus 99 oscillators truncated to d = 10, t_n = 0.5, omega_n = 1),
chi_max = 100, RRSVD with p = 10, q = 2, per-bond discarded weight
<= 1e-10, dt = 0.05, symmetric Trotter steps from |up>|0...0>.  One step is
three sweeps (even, odd, even bonds) over all 16 chains = 2384 bond updates.
W warm-up steps, then K timed steps, continue one run of W + K = 200 steps
by default, so the timed region covers the whole evolution.

The JSON line also carries:
* roofline   -- the kernel kind with the largest event time in the timed
                region; algorithmic flops from the recorded bond dimensions
                of every problem, divided by its event-timed duration;
* cpu_baseline -- the FP64 CPU oracle (full-SVD TEBD of chain 0 of the same
                workload) timed on the host for a bounded sample;
* full_svd   -- the same TEBD steps with the vendor full SVD
                (torch.linalg.svd) in a torch-only comparator on this GPU;
* batched_rrsvd -- the 256-matrix standalone RRSVD workload (sizes
                256..2048, s_i = exp(-i/25), k = 64, p = 10, q = 2);
* mixed_precision -- the spin-boson workload at chi_max = 128 with the
                sketch and power-iteration GEMMs in complex FP32, beside the
                FP64 path on the same inputs (errors of lambda and <sigma_z>);
* adjoint    -- d<Z_0(T)>/dJ_b of the XX chain with random fields (N = 40,
                chi_max = 64, 50 steps of dt = 0.02, checkpoints every 10
                steps): time per gradient and its error against the stored
                references (exact-SVD reverse mode, central differences,
                free fermions).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 256 MiB device buffer three times (the known-size kernel "
                         "that scales the HBM byte counters) and exit")
    ap.add_argument("--steps", type=int, default=190)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--chains", type=int, default=16)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--full-svd-steps", type=int, default=-1,
                    help="steps of the torch full-SVD comparator (-1: same as --steps)")
    ap.add_argument("--full-svd-seconds", type=float, default=90.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-svd", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--mixed-steps", type=int, default=100)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--rank", choices=("adaptive", "fixed"), default="adaptive",
                    help="rank of the timed run: two-stage adaptive (k1 from the bond dimension, "
                         "k = chi_max when needed) or fixed k = chi_max")
    ap.add_argument("--no-other-rank", action="store_true",
                    help="skip the run with the other rank mode")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# algorithmic flop counts (complex arithmetic: one multiply-add = 8 flops)
def sketch_flops(m, n, l):
    return 8.0 * m * n * l


def qr_flops(rows, l):
    # Householder factorisation plus explicit thin Q, complex: 2 x 4 (2 r l^2 - 2 l^3 / 3)
    return 16.0 * rows * l * l - 16.0 / 3.0 * l ** 3


def theta_gate_flops(dl, dr, cl, cm, cr):
    return 8.0 * (dl * cl * cm * dr * cr + (dl * dr) ** 2 * cl * cr)


def sweep_problems(chi_row, dims, parity, chi_max, p, adaptive):
    """(dl, dr, cl, cm, cr, m, n, l) of every bond of one chain in a sweep.

    l is the sketch width of the pass that every bond runs: with the
    adaptive rank the first stage's k1 + p, k1 = chi_m + max(4, ceil(chi_m / 2))
    capped by chi_max (the few bonds that need the fixed-rank second stage
    add work that is not counted); otherwise chi_max + p.  Both capped by
    m and n."""
    out = []
    for b in range(parity, len(dims) - 1, 2):
        cl, cm, cr = int(chi_row[b]), int(chi_row[b + 1]), int(chi_row[b + 2])
        dl, dr = dims[b], dims[b + 1]
        m, n = dl * cl, dr * cr
        k = min(chi_max, cm + max(4, (cm + 1) // 2)) if adaptive else chi_max
        out.append((dl, dr, cl, cm, cr, m, n, min(k + p, m, n)))
    return out


def qr_bytes(rows, l, with_r=False):
    """HBM bytes a QR must move: read the rows x l sketch, write the thin Q
    (and the l x l R factor)."""
    return 16.0 * (2 * rows * l + (l * l if with_r else 0))


def kind_flops(chi_hist, parities, dims, chi_max, p, q, adaptive):
    """Algorithmic flops per profiled kernel kind over the recorded sweeps,
    and the QR launches' algorithmic bytes (key "qr_bytes", both QR kinds)."""
    tot = {"theta_gate": 0.0, "sketch_A_Omega": 0.0, "sketch_AH_Q": 0.0, "sketch_A_Qt": 0.0,
           "qr": 0.0, "qr_with_r": 0.0, "qr_bytes": 0.0}
    for chi, parity in zip(chi_hist, parities):
        for c in range(chi.shape[0]):
            for (dl, dr, cl, cm, cr, m, n, l) in sweep_problems(chi[c], dims, parity, chi_max, p,
                                                                adaptive):
                tot["theta_gate"] += theta_gate_flops(dl, dr, cl, cm, cr)
                tot["sketch_A_Omega"] += sketch_flops(m, n, l)
                tot["sketch_AH_Q"] += (q + 1) * sketch_flops(m, n, l)
                tot["sketch_A_Qt"] += q * sketch_flops(m, n, l)
                tot["qr"] += (q + 1) * qr_flops(m, l) + q * qr_flops(n, l)
                tot["qr_with_r"] += qr_flops(n, l)
                tot["qr_bytes"] += ((q + 1) * qr_bytes(m, l) + q * qr_bytes(n, l)
                                    + qr_bytes(n, l, with_r=True))
    return tot


COPY_PROBE_BYTES = 256 << 20
# HBM bytes of the QR kernels from rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE runs, scaled by the same counters on a copy of known size);
# used only while the QR source still matches the one the counters saw
QR_TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "qr_hbm_traffic_counters.txt")
QR_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1504_00992_amd",
                         "csrc", "factor.hip")


def code_digest(path):
    """sha256 of a C++ source with comments and white space removed, so that
    a change to the comments alone keeps the digest (and the counters)."""
    import hashlib
    import re
    text = open(path, encoding="utf-8").read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return hashlib.sha256(re.sub(r"\s+", "", text).encode()).hexdigest()


def qr_traffic():
    """Bytes per QR launch from the committed counter summary, or None when
    it is absent or was taken on another version of the QR code."""
    try:
        lines = open(QR_TRAFFIC_FILE).read().splitlines()
        digest = code_digest(QR_SOURCE)
    except OSError:
        return None
    fields = dict(l[2:].split(": ", 1) for l in lines if l.startswith("# ") and ": " in l)
    if fields.get("factor.hip code sha256") != digest:
        return None
    try:
        return float(fields["bytes per qr launch"])
    except (KeyError, ValueError):
        return None


KIND_BOUND = {"theta_gate": "mfma", "sketch_A_Omega": "mfma", "sketch_AH_Q": "mfma",
              "sketch_A_Qt": "mfma", "qr": "alu", "qr_with_r": "alu"}


def roofline(prof, flops):
    """Roofline entry for the kind with the largest event time."""
    kind = max(prof, key=lambda k: prof[k][0])
    ms, launches = prof[kind]
    entry = {"kernel": kind, "launches": launches, "event_ms_total": round(ms, 3),
             "avg_launch_us": round(1e3 * ms / launches, 2) if launches else None}
    if kind in ("qr", "qr_with_r", "small_svd"):
        entry["note"] = ("one launch = every size class the batch reaches, run side by side; "
                         "rocprofv3 lists the class kernels (k_qr_reg<512, 8, piv>, ...) separately")
    if kind in flops and ms > 0:
        ach = flops[kind] / (ms * 1e-3) / 1e12
        entry.update({"bound": KIND_BOUND[kind], "achieved": round(ach, 4),
                      "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                      "frac": round(ach / PEAK_FP64_TFLOPS, 5), "traffic": None})
        if kind == "qr":
            nl = launches + (prof["qr_with_r"][1] if "qr_with_r" in prof else 0)
            if nl and "qr_bytes" in flops:
                # per launch of either QR kind, as the counters are taken
                entry["algorithmic_bytes"] = round(flops["qr_bytes"] / nl)
            t = qr_traffic()
            if t is not None:
                entry["traffic"] = round(t)
                entry["traffic_note"] = ("HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by "
                                         "a copy of known size): " + os.path.basename(QR_TRAFFIC_FILE))
    else:
        entry.update({"bound": "alu", "achieved": None, "peak": PEAK_FP64_TFLOPS,
                      "unit": "TFLOP/s", "frac": None, "traffic": None,
                      "note": "iterative kernel: no fixed algorithmic flop count"})
    return entry


# ---------------------------------------------------------------------------
def run_gpu_tebd(args, torch, api, models, adaptive, prof_on=True):
    N, d, chi_max, p, q = 100, 10, 100, 10, 2
    dims, hb = models.spin_boson(N, d, 1.0, 0.5, 1.0, 0.5)
    mps = api.DeviceMPS.product_state(args.chains, dims, [0] * N, chi_max)
    drv = api.TEBD(mps, hb, 0.05, chi_max, p=p, q=q, trunc_eps=1e-10, seed=1504,
                   adaptive=2 if adaptive else 0)
    for _ in range(args.warmup):
        drv.step()
    torch.cuda.synchronize()
    # the profiled pass also records every sweep's bond dimensions (for the
    # algorithmic flop counts of the roofline)
    chi_hist = torch.empty((3 * args.steps, args.chains, N + 1), dtype=torch.int32, device="cuda")
    parities = []
    api._lib.tebd_profile_enable(prof_on)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = 0
    for _ in range(args.steps):
        for parity, gates in ((0, drv.g_half), (1, drv.g_full), (0, drv.g_half)):
            if prof_on:
                chi_hist[k].copy_(mps.chi)
            parities.append(parity)
            drv.sweep(parity, gates)
            k += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = api._lib.tebd_profile_read() if prof_on else {}
    api._lib.tebd_profile_enable(False)
    status = drv.ws.status.cpu().numpy()
    return dict(seconds=t1 - t0, prof=prof, chi_hist=chi_hist.cpu().numpy(), parities=parities,
                dims=dims, hb=hb, chi_final=mps.chi.cpu().numpy(), status=status)


def updates_per_step(n_sites):
    even = (n_sites - 1 + 1) // 2
    odd = (n_sites - 1) // 2
    return 2 * even + odd


def full_svd_tebd(args, torch, models, dims, hb, warmup, steps):
    """torch-only TEBD with torch.linalg.svd (full SVD) on the same workload.

    Runs `warmup` untimed steps, then times up to `steps` steps (stopping
    early after --full-svd-seconds, which only flatters the comparator since
    later steps carry larger bonds)."""
    N, chi_max, eps, floor_ = len(dims), 100, 1e-10, 1e-14
    dev = "cuda"
    nch = args.chains
    dmax = max(dims)
    gam = torch.zeros((nch, N, dmax, chi_max, chi_max), dtype=torch.complex128, device=dev)
    lam = torch.zeros((nch, N - 1, chi_max), dtype=torch.float64, device=dev)
    gam[:, :, 0, 0, 0] = 1.0
    lam[:, :, 0] = 1.0
    chi = [[1] * (N + 1) for _ in range(nch)]
    gh = [torch.from_numpy(models.propagator(h, 0.025)).to(dev) for h in hb]
    gf = [torch.from_numpy(models.propagator(h, 0.05)).to(dev) for h in hb]

    def bond(b, g):
        groups = {}
        for c in range(nch):
            groups.setdefault((chi[c][b], chi[c][b + 1], chi[c][b + 2]), []).append(c)
        dl, dr = dims[b], dims[b + 1]
        for (cl, cm, cr), chains in groups.items():
            idx = torch.tensor(chains, device=dev)
            gk = gam[idx, b, :dl, :cl, :cm]
            gk1 = gam[idx, b + 1, :dr, :cm, :cr]
            ll = lam[idx, b - 1, :cl] if b >= 1 else torch.ones((len(chains), cl), dtype=torch.float64, device=dev)
            lm = lam[idx, b, :cm]
            lr = lam[idx, b + 1, :cr] if b + 1 <= N - 2 else torch.ones((len(chains), cr), dtype=torch.float64, device=dev)
            left = (gk * ll[:, None, :, None] * lm[:, None, None, :]).contiguous()
            right = (gk1 * lr[:, None, None, :]).contiguous()
            th = torch.einsum("biag,bjgc->bijac", left, right).reshape(len(chains), dl * dr, cl * cr)
            tt = torch.matmul(g, th)
            a = tt.reshape(len(chains), dl, dr, cl, cr).permute(0, 1, 3, 2, 4).reshape(len(chains), dl * cl, dr * cr)
            u, s, vh = torch.linalg.svd(a, full_matrices=False)
            s2 = (s * s).cpu().numpy()
            for j, c in enumerate(chains):
                tot = s2[j].sum()
                tails = (tot - s2[j].cumsum()) / tot
                ok = [i for i in range(len(tails)) if tails[i] <= eps]
                cp = min(chi_max, (ok[0] + 1) if ok else len(tails))
                nrm = float(s2[j][:cp].sum()) ** 0.5
                inv_l = torch.where(ll[j] > floor_, 1.0 / ll[j], torch.zeros_like(ll[j]))
                inv_r = torch.where(lr[j] > floor_, 1.0 / lr[j], torch.zeros_like(lr[j]))
                gam[c, b, :, :, :] = 0
                gam[c, b + 1, :, :, :] = 0
                gam[c, b, :dl, :cl, :cp] = u[j, :, :cp].reshape(dl, cl, cp) * inv_l[None, :, None]
                gam[c, b + 1, :dr, :cp, :cr] = vh[j, :cp, :].reshape(cp, dr, cr).permute(1, 0, 2) * inv_r[None, None, :]
                lam[c, b, :] = 0
                lam[c, b, :cp] = s[j, :cp] / nrm
                chi[c][b + 1] = cp

    def step():
        for parity, gs in ((0, gh), (1, gf), (0, gh)):
            for b in range(parity, N - 1, 2):
                bond(b, gs[b])

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    last = t0
    for _ in range(steps):
        step()
        done += 1
        torch.cuda.synchronize()
        now = time.perf_counter()
        if now - last > 20.0:
            _progress(f"full-SVD comparator: {done} steps, {now - t0:.0f} s")
            last = now
        if now - t0 > args.full_svd_seconds:
            break
    torch.cuda.synchronize()
    return done, time.perf_counter() - t0


def cpu_oracle_baseline(args, dims, budget_s):
    """FP64 oracle TEBD (full LAPACK SVD) of chain 0, bounded by wall time."""
    import numpy as np
    from oracle import models as om, mps as omps
    try:
        from threadpoolctl import threadpool_info
        threads = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
    except Exception:
        threads = 1
    N = len(dims)
    _, hb = om.spin_boson_chain(N, dims[1], 1.0, 0.5, 1.0, 0.5)
    cache = {}

    def gfn(b, tau):
        key = (b, tau)
        if key not in cache:
            cache[key] = om.gate(hb[b], tau)
        return cache[key]
    m = omps.basis_product_state(dims, [0] * N)
    drv = omps.TEBD(m, gfn, 0.05, 100, 1e-10, method="full")
    for b in range(N - 1):  # gates outside the timed sample
        gfn(b, 0.025), gfn(b, 0.05)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < budget_s:
        drv.step()
        steps += 1
    dt = time.perf_counter() - t0
    upd = steps * updates_per_step(N)
    return {"value": round(upd / dt, 2), "unit": "bond updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"chain 0 of the same workload, steps 1..{steps} of the run "
                      f"({upd} bond updates, {dt:.1f} s), FP64 full LAPACK SVD per bond"}


def batched_rrsvd(torch, api, wl):
    sizes = wl.batched_rrsvd_sizes()
    mats = wl.batched_rrsvd_matrices_device(sizes)
    from paper_1504_00992_amd import _lib
    api.rrsvd_truncate(mats, 64, 10, 2, 1e-10, 1504, 0)  # warm-up (workspace, code)
    torch.cuda.synchronize()
    reps = 3
    _lib.tebd_profile_enable(True)
    t0 = time.perf_counter()
    for r in range(reps):
        out = api.rrsvd_truncate(mats, 64, 10, 2, 1e-10, 1504, r + 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = _lib.tebd_profile_read()
    _lib.tebd_profile_enable(False)
    l = 74
    f_sk = sum(sketch_flops(n, n, l) for n in sizes)
    sk_ms = sum(prof.get(k, (0.0, 0))[0] for k in ("sketch_A_Omega", "sketch_AH_Q", "sketch_A_Qt")) / reps
    sk_fl = 6 * f_sk
    ach = sk_fl / (sk_ms * 1e-3) / 1e12 if sk_ms > 0 else None
    return {"metric": "RRSVD truncations/s", "value": round(len(sizes) * reps / (t1 - t0), 2),
            "ms_per_batch": round(1e3 * (t1 - t0) / reps, 3),
            "config": {"workload": "256 complex128 square matrices, n in {256,512,1024,2048}, "
                                   "s_i=exp(-i/25), k=64, p=10, q=2, one call"},
            "sketch_gemms": {"bound": "mfma", "achieved": round(ach, 3) if ach else None,
                             "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                             "frac": round(ach / PEAK_FP64_TFLOPS, 4) if ach else None,
                             "ms_per_batch": round(sk_ms, 3)},
            "phase_ms_per_batch": {k: round(v[0] / reps, 3) for k, v in prof.items()}}


def _spin_z(torch, gamma, lam, chains):
    from paper_1504_00992_amd import gradient
    z = torch.zeros((gamma.shape[2], gamma.shape[2]), dtype=torch.complex128, device="cuda")
    z[0, 0], z[1, 1] = 1.0, -1.0
    return [float(gradient.expectation(gamma[c], lam[c], z, 0).item()) for c in range(chains)]


def mixed_precision(args, torch, api, models):
    """Spin-boson chains at chi_max = 128: complex FP32 sketch / power GEMMs
    (precision = 1) against the FP64 path on the same inputs and seeds."""
    import numpy as np
    N, d, chi_max, steps = 100, 10, 128, args.mixed_steps
    dims, hb = models.spin_boson(N, d, 1.0, 0.5, 1.0, 0.5)
    out = {}
    for prec in (0, 1):
        mps = api.DeviceMPS.product_state(args.chains, dims, [0] * N, chi_max)
        drv = api.TEBD(mps, hb, 0.05, chi_max, p=10, q=2, trunc_eps=1e-10, seed=1504,
                       precision=prec, adaptive=2)
        for _ in range(min(args.warmup, 2)):
            drv.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            drv.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out[prec] = dict(sec=t1 - t0, chi=mps.chi.cpu().numpy(), lam=mps.lam.cpu().numpy(),
                         z=_spin_z(torch, mps.gamma, mps.lam, args.chains))
    same = bool(np.array_equal(out[0]["chi"], out[1]["chi"]))
    lam_err = float(np.max(np.abs(out[0]["lam"] - out[1]["lam"]))) if same else None
    z_err = float(np.max(np.abs(np.array(out[0]["z"]) - np.array(out[1]["z"]))))
    per = updates_per_step(N) * args.chains * steps
    return {"config": {"workload": f"{args.chains} spin-boson chains N=100 d=10, chi_max=128, "
                                   f"dt=0.05, {steps} steps after warm-up, adaptive rank"},
            "mixed_value": round(per / out[1]["sec"], 2), "fp64_value": round(per / out[0]["sec"], 2),
            "unit": "bond updates/s",
            "bond_dims_identical": same,
            "max_abs_lambda_diff": lam_err,
            "max_abs_sigma_z_diff": z_err,
            "reference": "the FP64 path on the same inputs (its own parity with the CPU oracle "
                         "is checked in the GPU tests)"}


def adjoint_gradient(torch, api, models, wl, reps=3):
    """Time per gradient of <Z_0(T)> w.r.t. the 39 couplings (XX + fields, N=40)."""
    import numpy as np
    from paper_1504_00992_amd import gradient
    n, steps, dt, chi_max = 40, 50, 0.02, 64
    J, h = wl.xx_couplings(n, seed=1504)
    dims, hb = models.xx_chain(J, h)
    hop = 0.5 * (np.kron(models.PAULI_X, models.PAULI_X) + np.kron(models.PAULI_Y, models.PAULI_Y))
    g_half = torch.from_numpy(models.gate_stack(dims, hb, 0.5 * dt)).cuda()
    g_full = torch.from_numpy(models.gate_stack(dims, hb, dt)).cuda()
    z = torch.tensor([[1.0, 0.0], [0.0, -1.0]], dtype=torch.complex128, device="cuda")
    timings = []
    grad = None
    for rep in range(reps + 1):
        mps = api.DeviceMPS.product_state(1, dims, wl.neel_levels(n), chi_max)
        drv = gradient.CheckpointedTEBD(mps, g_half, g_full, chi_max, 10, 2, 1e-10, 1504,
                                        adaptive=2, checkpoint=10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        drv.forward(steps)
        gam = mps.gamma[0].clone().requires_grad_(True)
        lam = mps.lam[0].clone().requires_grad_(True)
        val = gradient.expectation(gam, lam, z, 0)
        val.backward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gb = torch.zeros_like(mps.gamma)
        lb = torch.zeros_like(mps.lam)
        gb[0] = gam.grad
        lb[0] = lam.grad
        gh, gf, _, _ = drv.backward(gb, lb)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        gh, gf = gh.cpu().numpy(), gf.cpu().numpy()
        grad = np.array([gradient.coupling_gradient(gh[b], hb[b], 0.5 * dt, hop)
                         + gradient.coupling_gradient(gf[b], hb[b], dt, hop) for b in range(n - 1)])
        t3 = time.perf_counter()
        if rep > 0:  # the first is a warm-up
            timings.append((t1 - t0, t2 - t1, t3 - t2))
    ref = np.loadtxt(os.path.join(ROOT, "tests", "golden", "xx_n40_gradient.txt"))
    scale = float(np.max(np.abs(ref[:, 3])))
    fw, bw, host = (float(np.median([t[i] for t in timings])) for i in range(3))
    return {"config": {"workload": "XX chain + random fields, N=40, J_b~U[0.8,1.2], h_i~U[-1,1], "
                                   "Neel start, 50 steps dt=0.02, chi_max=64, w<=1e-10, "
                                   "checkpoint every 10 steps; gradient of <Z_0(T=1)> w.r.t. "
                                   "all 39 J_b"},
            "ms_per_gradient": round(1e3 * (fw + bw + host), 2),
            "forward_ms": round(1e3 * fw, 2), "reverse_ms": round(1e3 * bw, 2),
            "host_frechet_ms": round(1e3 * host, 2),
            "rel_err_vs_exact_svd_reverse": float(np.max(np.abs(grad - ref[:, 2])) / scale),
            "rel_err_vs_finite_differences": float(np.max(np.abs(grad - ref[:, 3])) / scale),
            "rel_err_vs_free_fermions": float(np.max(np.abs(grad - ref[:, 4])) / scale),
            "note": "errors relative to max|dL/dJ_b|; references in tests/golden/xx_n40_gradient.txt"}


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU layout is "
              f"described in DESIGN.md and not launched here.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": COPY_PROBE_BYTES, "copies": 3}))
        return
    from paper_1504_00992_amd import api, models, _lib
    import workloads as wl
    _lib.load()

    adaptive = args.rank == "adaptive"
    # value: the run without per-phase events (each event record adds a gap
    # between launches); phase times and the roofline: the same run again
    # with HIP events around every phase
    res = run_gpu_tebd(args, torch, api, models, adaptive, prof_on=False)
    _progress(f"timed TEBD run: {res['seconds']:.2f} s")
    profd = run_gpu_tebd(args, torch, api, models, adaptive, prof_on=True)
    _progress(f"profiled TEBD run: {profd['seconds']:.2f} s")
    N = 100
    per_step = updates_per_step(N) * args.chains
    total_updates = per_step * args.steps
    sec = res["seconds"]
    value = total_updates / sec
    flops = kind_flops(profd["chi_hist"], profd["parities"], profd["dims"], 100, 10, 2, adaptive)
    prof = profd["prof"]
    line = {
        "metric": "TEBD bond updates/s, RRSVD vs full SVD on 1 GPU at <=1e-10 trunc err",
        "value": round(value, 2),
        "unit": "bond updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * sec / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 (f64)",
        "data": "synthetic",
        "config": {"workload": "batched TEBD sweep: 16 chain-mapped spin-boson chains, N=100 "
                               "(spin + 99 oscillators, d=10), t_n=0.5, w_n=1, dt=0.05, chi_max=100, "
                               "RRSVD p=10 q=2, w<=1e-10 per bond",
                   "rank": ("two-stage adaptive: k1 = chi + max(4, chi/2), k = chi_max when the "
                            "Frobenius residual needs it (second pass skipped on the host when no "
                            "bond needs it)" if adaptive else "fixed k = chi_max"),
                   "chains": args.chains, "bond_updates_per_step": per_step,
                   "chi_final_max": int(res["chi_final"].max()),
                   "status_bits_seen": sorted(set(int(x) for x in np.unique(res["status"])))},
        "phase_ms": {k: round(v[0], 3) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])},
        "phase_launches": {k: int(v[1]) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])},
        "profiled_ms_per_step": round(1e3 * profd["seconds"] / args.steps, 4),
        "roofline": roofline(prof, flops),
    }
    line["roofline"]["measured"] = ("HIP events around every phase in a second pass of the same "
                                    "timed steps (same inputs, same kernels); value is timed "
                                    "without events")
    if not args.no_other_rank:
        other = run_gpu_tebd(args, torch, api, models, not adaptive, prof_on=False)
        oval = total_updates / other["seconds"]
        _progress(f"other rank mode: {other['seconds']:.2f} s")
        line["other_rank_mode"] = {
            "rank": "fixed k = chi_max" if adaptive else "two-stage adaptive",
            "value": round(oval, 2), "unit": "bond updates/s",
            "ms_per_step": round(1e3 * other["seconds"] / args.steps, 4),
            "chi_final_max": int(other["chi_final"].max())}
    if not args.no_full_svd:
        nsteps = args.steps if args.full_svd_steps < 0 else args.full_svd_steps
        done, fsec = full_svd_tebd(args, torch, models, res["dims"], res["hb"], args.warmup, nsteps)
        fval = done * per_step / fsec if fsec > 0 else None
        _progress(f"full-SVD comparator: {done} steps in {fsec:.1f} s")
        line["full_svd"] = {"value": round(fval, 2), "unit": "bond updates/s",
                            "steps": done, "seconds": round(fsec, 2),
                            "note": "torch.linalg.svd (vendor full SVD) in a torch-only TEBD step on "
                                    "the same GPU, same warm-up, timed steps after it"}
        line["speedup_vs_full_svd"] = round(value / fval, 3) if fval else None
    if not args.no_batched:
        line["batched_rrsvd"] = batched_rrsvd(torch, api, wl)
        _progress("batched RRSVD done")
    if not args.no_mixed:
        line["mixed_precision"] = mixed_precision(args, torch, api, models)
        _progress("mixed precision done")
    if not args.no_adjoint:
        line["adjoint"] = adjoint_gradient(torch, api, models, wl)
        _progress("adjoint done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_oracle_baseline(args, res["dims"], args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
