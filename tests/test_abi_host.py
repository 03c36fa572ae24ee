"""CPU-only checks of the C interface: symbols, argument validation, sizes.

No kernel is launched: every call here returns from host-side validation
before anything is enqueued (or only computes a workspace size).
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1504_00992_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tebd_rrsvd.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:tebd_status|const char\*|int32_t)\s+(\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = _lib.load()
    names = _declared_functions()
    assert set(names) == set(_lib.EXPORTED)
    for name in names:
        assert hasattr(lib, name), name
    assert "gfx950" in _lib.tebd_version()


def test_struct_layouts_match_header():
    # tebd_params: 4 x int32, 2 x double, uint64, 2 x uint32 = 48 bytes
    assert ctypes.sizeof(_lib.TebdParams) == 48
    assert _lib.TebdParams.trunc_eps.offset == 16 and _lib.TebdParams.seed.offset == 32
    assert _lib.TebdParams.adaptive.offset == 44
    # tebd_mps: 4 x int32 then 4 pointers
    assert ctypes.sizeof(_lib.TebdMps) == 48 and _lib.TebdMps.d.offset == 16


def _ws(prm, m, n):
    return _lib.tebd_workspace_size(prm, m=m, n=n)


def test_workspace_size_and_validation():
    prm = _lib.params(64, 10, 2)
    small = _ws(prm, [256], [256])
    big = _ws(prm, [2048], [2048])
    assert 0 < small < big
    two = _ws(prm, [256, 2048], [256, 2048])
    assert two > big
    with pytest.raises(_lib.TebdError) as e:
        _ws(_lib.params(0), [8], [8])
    assert e.value.status == _lib.TEBD_ERR_ARG and "chi_max" in str(e.value)
    with pytest.raises(_lib.TebdError) as e:
        _ws(prm, [0], [8])
    assert e.value.status == _lib.TEBD_ERR_SHAPE
    bad = _lib.params(8, 10, 2)
    bad.adaptive = 4
    with pytest.raises(_lib.TebdError):
        _ws(bad, [8], [8])
    bad = _lib.params(8, 0, 2, adaptive=3)  # the Accuracy Check probes p >= 1 columns
    with pytest.raises(_lib.TebdError) as e:
        _ws(bad, [8], [8])
    assert "p >= 1" in str(e.value)
    with pytest.raises(_lib.TebdError) as e:  # rows beyond the supported 8192
        _ws(prm, [8193], [8])
    assert e.value.status == _lib.TEBD_ERR_SHAPE
    with pytest.raises(_lib.TebdError) as e:
        _ws(_lib.params(8, trunc_eps=0.0, adaptive=1), [8], [8])
    assert "trunc_eps" in str(e.value)
    with pytest.raises(_lib.TebdError) as e:
        _ws(_lib.params(8, q=-1), [8], [8])
    assert "q" in str(e.value)


def _mps_struct(n_chains=2, n_sites=6, d_max=2, chi_max=8, null=None):
    fake = 0x100000  # never dereferenced: validation fails or only sizes are computed
    ptrs = {"d": fake, "gamma": fake, "lambda_": fake, "chi": fake}
    if null:
        ptrs[null] = None
    return _lib.TebdMps(n_chains, n_sites, d_max, chi_max, ptrs["d"], ptrs["gamma"],
                        ptrs["lambda_"], ptrs["chi"])


def test_sweep_workspace_scales_with_capacity():
    prm = _lib.params(8)
    a = _lib.tebd_workspace_size(prm, mps=_mps_struct())
    b = _lib.tebd_workspace_size(prm, mps=_mps_struct(n_chains=4))
    assert 0 < a < b
    with pytest.raises(_lib.TebdError) as e:
        _lib.tebd_workspace_size(_lib.params(16), mps=_mps_struct(chi_max=8))
    assert e.value.status == _lib.TEBD_ERR_SHAPE


@pytest.mark.parametrize("null", ["d", "gamma", "lambda_", "chi"])
def test_sweep_rejects_null_mps_arrays(null):
    prm = _lib.params(8)
    st = _lib.tebd_sweep(_mps_struct(null=null), 0x100000, 0, 0, prm, 0x100000, 0x100000, 0x100000,
                         1 << 30, None)
    assert st == _lib.TEBD_ERR_ARG
    assert null.rstrip("_") in _lib.tebd_last_error()


def test_sweep_rejects_bad_arguments_before_enqueue():
    prm = _lib.params(8)
    mps = _mps_struct()
    # parity out of range
    assert _lib.tebd_sweep(mps, 0x100000, 0, 2, prm, 0x100000, 0x100000, 0x100000, 1 << 30,
                           None) == _lib.TEBD_ERR_ARG
    assert "parity" in _lib.tebd_last_error()
    # null gates
    assert _lib.tebd_sweep(mps, None, 0, 0, prm, 0x100000, 0x100000, 0x100000, 1 << 30,
                           None) == _lib.TEBD_ERR_ARG
    # workspace too small / misaligned / missing
    need = _lib.tebd_workspace_size(prm, mps=mps)
    assert _lib.tebd_sweep(mps, 0x100000, 0, 0, prm, 0x100000, 0x100000, 0x100000, need - 1,
                           None) == _lib.TEBD_ERR_WORKSPACE
    assert _lib.tebd_sweep(mps, 0x100000, 0, 0, prm, 0x100000, 0x100000, 0x100008, need,
                           None) == _lib.TEBD_ERR_WORKSPACE
    assert _lib.tebd_sweep(mps, 0x100000, 0, 0, prm, 0x100000, 0x100000, None, need,
                           None) == _lib.TEBD_ERR_WORKSPACE
    # bond update: bond out of range, chain out of range
    assert _lib.tebd_bond_update(mps, 0, 5, 0x100000, prm, 0x100000, 0x100000, 0x100000, need,
                                 None) == _lib.TEBD_ERR_ARG
    assert _lib.tebd_bond_update(mps, 2, 0, 0x100000, prm, 0x100000, 0x100000, 0x100000, need,
                                 None) == _lib.TEBD_ERR_ARG
    assert "chain" in _lib.tebd_last_error()


def test_rrsvd_rejects_bad_arguments_before_enqueue():
    prm = _lib.params(4)
    f = 0x100000
    args = dict(m=[8], n=[6], a_ptrs=[f], lda=[6], omega_ptrs=None, prm=prm, u_ptrs=[f], ldu=4,
                s_ptrs=[f], vh_ptrs=[f], ldvh=6, chi_kept_ptr=f, disc_ptr=f, status_ptr=f,
                ws_ptr=f, ws_bytes=1 << 30, stream=None)

    def call(**kw):
        a = dict(args)
        a.update(kw)
        return _lib.rrsvd_truncate(**a)

    assert call(lda=[5]) == _lib.TEBD_ERR_SHAPE and "lda" in _lib.tebd_last_error()
    assert call(ldu=3) == _lib.TEBD_ERR_SHAPE
    assert call(ldvh=5) == _lib.TEBD_ERR_SHAPE
    assert call(a_ptrs=[None]) == _lib.TEBD_ERR_ARG
    assert call(chi_kept_ptr=None) == _lib.TEBD_ERR_ARG
    assert call(ws_bytes=16) == _lib.TEBD_ERR_WORKSPACE
    assert call(ws_ptr=f + 8) == _lib.TEBD_ERR_WORKSPACE
    assert call(m=[0]) == _lib.TEBD_ERR_SHAPE
    assert call(omega_ptrs=[None]) == _lib.TEBD_ERR_ARG
    assert call(prm=_lib.params(4, adaptive=1)) == _lib.TEBD_ERR_ARG
    assert "TEBD entry points" in _lib.tebd_last_error()


def test_product_gates_match_oracle_gates():
    # The product builds its gates with its own code; both must agree.
    from oracle import models as om
    import workloads as wl
    from paper_1504_00992_amd import models as pm
    dims_o, hb_o = om.spin_boson_chain(5, 4)
    dims_p, hb_p = pm.spin_boson(5, 4)
    assert dims_o == dims_p
    for a, b in zip(hb_o, hb_p):
        assert np.allclose(a, b, atol=1e-14)
    gates = pm.gate_stack(dims_p, hb_p, 0.05)
    for k, h in enumerate(hb_o):
        g = om.gate(h, 0.05)
        assert np.allclose(gates[k, :g.shape[0], :g.shape[0]], g, atol=1e-13)
    J, h = wl.xx_couplings(6, seed=2)
    for a, b in zip(om.xx_field(J, h)[1], pm.xx_chain(J, h)[1]):
        assert np.allclose(a, b, atol=1e-14)
    for a, b in zip(om.tfim(6, 0.8, 1.1)[1], pm.transverse_ising(6, 0.8, 1.1)[1]):
        assert np.allclose(a, b, atol=1e-14)


def test_adjoint_entry_points_validate_before_enqueue():
    prm = _lib.params(8)
    mps = _mps_struct()
    f = 0x100000
    tb = _lib.tebd_tape_size(mps, prm)
    assert tb > 0
    need = _lib.tebd_adjoint_workspace_size(mps, prm)
    assert need >= _lib.tebd_workspace_size(prm, mps=mps)
    lib = _lib.load()

    def rec(**kw):
        a = dict(gates=f, parity=0, tape=f, tape_bytes=tb, ws=f, ws_bytes=need)
        a.update(kw)
        return _lib.tebd_sweep_record(mps, a["gates"], 0, a["parity"], prm, f, f, a["tape"],
                                      a["tape_bytes"], a["ws"], a["ws_bytes"], None)
    assert rec(tape=None) == _lib.TEBD_ERR_ARG and "tape" in _lib.tebd_last_error()
    assert rec(tape=f + 8) == _lib.TEBD_ERR_WORKSPACE
    assert rec(tape_bytes=tb - 1) == _lib.TEBD_ERR_WORKSPACE
    assert rec(parity=3) == _lib.TEBD_ERR_ARG

    def adj(**kw):
        a = dict(tape=f, tape_bytes=tb, gb=f, lb=f, gbar=f, status=f, ws=f, ws_bytes=need,
                 parity=1)
        a.update(kw)
        return _lib.tebd_sweep_adjoint(mps, f, 0, a["parity"], prm, a["tape"], a["tape_bytes"],
                                       a["gb"], a["lb"], a["gbar"], a["status"], a["ws"],
                                       a["ws_bytes"], None)
    assert adj(tape=None) == _lib.TEBD_ERR_ARG
    assert adj(gb=None) == _lib.TEBD_ERR_ARG and "gamma_bar" in _lib.tebd_last_error()
    assert adj(lb=None) == _lib.TEBD_ERR_ARG and "lambda_bar" in _lib.tebd_last_error()
    assert adj(gbar=None) == _lib.TEBD_ERR_ARG and "gate_bar" in _lib.tebd_last_error()
    assert adj(status=None) == _lib.TEBD_ERR_ARG
    assert adj(tape_bytes=16) == _lib.TEBD_ERR_WORKSPACE
    assert adj(ws_bytes=need - 1) == _lib.TEBD_ERR_WORKSPACE
    assert adj(ws=f + 8) == _lib.TEBD_ERR_WORKSPACE
    assert adj(parity=-1) == _lib.TEBD_ERR_ARG
    # the tape grows with the chain batch
    assert _lib.tebd_tape_size(_mps_struct(n_chains=4), prm) == 2 * tb
    del lib


def test_propagator_derivative_matches_finite_differences():
    from paper_1504_00992_amd import gradient, models as pm
    gen = np.random.default_rng(4)
    h = gen.standard_normal((4, 4)) + 1j * gen.standard_normal((4, 4))
    h = h + h.conj().T
    h[0, 0] = h[1, 1]  # a near-degenerate pair is handled
    dh = gen.standard_normal((4, 4)) + 1j * gen.standard_normal((4, 4))
    dh = dh + dh.conj().T
    tau = 0.37
    got = gradient.propagator_derivative(h, tau, dh)
    fd = (pm.propagator(h + 1e-6 * dh, tau) - pm.propagator(h - 1e-6 * dh, tau)) / 2e-6
    assert np.max(np.abs(got - fd)) < 1e-9
    gbar = gen.standard_normal((4, 4)) + 1j * gen.standard_normal((4, 4))
    assert gradient.coupling_gradient(gbar, h, tau, dh) == pytest.approx(
        float(np.real(np.sum(gbar.conj() * fd))), abs=1e-8)


def test_noalloc_refuses_batches_beyond_its_scratch():
    # 4 problems of 4096 x 4096 at l = 110 need about 86 MB of scratch, more
    # than the 64 MiB static array: refused on the host, nothing enqueued
    # (the fake device pointers are never touched)
    lib = _lib.load()
    batch = 4
    m = [4096] * batch
    prm = _lib.params(100, 10, 2, 1e-10)
    fake = [0x1000 * (i + 1) for i in range(batch)]
    st = _lib.rrsvd_truncate_noalloc(m, m, fake, m, None, prm, fake, 100, fake, fake, 4096,
                                     0x1000, 0x1000, 0x1000, None)
    assert st == _lib.TEBD_ERR_WORKSPACE
    assert "64" in _lib.tebd_last_error() or "scratch" in _lib.tebd_last_error()


def test_autotune_cache_entries_and_json_round_trip(tmp_path):
    # the cache's bucket mapping and validation (host only), and a JSON file
    # written by the autotuner's save() loaded back into the library
    from paper_1504_00992_amd import autotune
    _lib.load()
    assert _lib.tebd_tune_set(0, 300, 50, 1) == _lib.TEBD_OK
    assert _lib.tebd_tune_get(0, 512, 64) == 1      # same bucket (<= 512, <= 64)
    assert _lib.tebd_tune_get(0, 256, 64) in (-1, 0, 1)
    assert _lib.tebd_tune_set(1, 300, 50, 1) == _lib.TEBD_ERR_ARG   # FP32 products: variant 0 only
    assert _lib.tebd_tune_set(0, 300, 70, 1) == _lib.TEBD_OK
    assert _lib.tebd_tune_get(0, 512, 80) == 1                      # width bucket (64, 80]
    assert _lib.tebd_tune_get(0, 512, 81) != 1                      # the next bucket, (80, 128]
    assert _lib.tebd_tune_set(0, 300, 70, 2) == _lib.TEBD_OK       # split-depth 16 x 16 tiles
    assert _lib.tebd_tune_get(0, 512, 80) == 2
    assert _lib.tebd_tune_set(0, 300, 70, 3) == _lib.TEBD_ERR_ARG
    assert _lib.tebd_tune_set(2, 1000, 110, 2) == _lib.TEBD_OK      # the TEBD sweep table
    assert _lib.tebd_tune_get(2, 1024, 128) == 2 and _lib.tebd_tune_get(0, 1024, 128) != 2
    assert _lib.tebd_tune_set(2, 1000, 110, -1) == _lib.TEBD_OK
    assert _lib.tebd_tune_set(3, 1000, 110, 0) == _lib.TEBD_ERR_ARG
    assert _lib.tebd_tune_set(0, 9000, 50, 0) == _lib.TEBD_ERR_SHAPE
    assert _lib.tebd_tune_set(0, 300, 300, 0) == _lib.TEBD_ERR_SHAPE
    assert _lib.tebd_tune_get(2, 10, 10) == -1
    path = autotune.save([{"precision": 0, "rows": 2048, "width": 128, "variant": 1},
                          {"precision": 0, "rows": 100, "width": 20, "variant": 0}],
                         str(tmp_path / "t.json"), "test")
    got = autotune.load(path)
    assert len(got) == 2
    assert _lib.tebd_tune_get(0, 1500, 100) == 1 and _lib.tebd_tune_get(0, 128, 32) == 0
    assert autotune.load(str(tmp_path / "absent.json")) == []
    for rows, width in ((300, 50), (300, 70), (1500, 100), (128, 32)):
        assert _lib.tebd_tune_set(0, rows, width, -1) == _lib.TEBD_OK
        assert _lib.tebd_tune_get(0, rows, width) == -1
