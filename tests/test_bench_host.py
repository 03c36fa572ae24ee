"""Host-side accounting of bench.py (no GPU): the sketch width the
algorithmic counts use, the QR byte count, and the rule that measured HBM
traffic is only reported for the QR source the counters were taken on."""
import importlib.util
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_sketch_width_adaptive_and_fixed():
    b = _bench()
    dims = [2, 10, 10, 10]
    chi = np.array([1, 2, 19, 14, 1])
    # bond 1: chi_m = 19 -> k1 = 19 + 10 = 29, l = k1 + p = 39 (m = 20 caps it)
    (dl, dr, cl, cm, cr, m, n, l), = b.sweep_problems(chi, dims, 1, 100, 10, True)[:1]
    assert (cl, cm, cr, m, n) == (2, 19, 14, 20, 140) and l == 20
    dims2 = [10, 10, 10, 10]
    chi2 = np.array([1, 19, 19, 14, 1])
    out = b.sweep_problems(chi2, dims2, 1, 100, 10, True)
    assert out[0][-1] == 29 + 10                  # adaptive: chi_m + ceil(chi_m / 2) + p
    assert b.sweep_problems(chi2, dims2, 1, 100, 10, False)[0][-1] == 110   # fixed: chi_max + p
    # small bonds use the margin 4: chi_m = 1 -> k1 = 5
    assert b.sweep_problems(np.array([1, 1, 1, 1, 1]), dims2, 0, 100, 10, True)[0][-1] == 10


def test_qr_bytes():
    b = _bench()
    assert b.qr_bytes(10, 3) == 16 * 2 * 10 * 3
    assert b.qr_bytes(10, 3, with_r=True) == 16 * (2 * 10 * 3 + 9)


def test_traffic_only_for_the_measured_source(tmp_path):
    b = _bench()
    src = tmp_path / "factor.hip"
    src.write_text("// some QR source\nint f() { return 1; }\n")
    digest = b.code_digest(str(src))
    summary = tmp_path / "qr_hbm_traffic_counters.txt"
    summary.write_text(f"# factor.hip code sha256: {digest}\n# bytes per qr launch: 1234\n")
    b.QR_SOURCE, b.QR_TRAFFIC_FILE = str(src), str(summary)
    assert b.qr_traffic() == 1234.0
    src.write_text("/* reworded */ int f()  {\n  return 1;  // comment\n}\n")  # comments only
    assert b.qr_traffic() == 1234.0
    src.write_text("int f() { return 2; }\n")  # the code changed since the counters
    assert b.qr_traffic() is None
    b.QR_TRAFFIC_FILE = str(tmp_path / "absent.txt")
    assert b.qr_traffic() is None
