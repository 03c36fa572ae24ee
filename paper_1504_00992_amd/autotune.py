"""Autotuner of the sketch products' tile shape (the library's autotune cache).

For each (largest rows, sketch width) bucket of the cache, a synthetic batch
of that shape is truncated with each tile variant of the sketch, power-
iteration and projection products (32 x 32 or 64 x 64 output tiles, or
16 x 16 tiles split over the contraction depth), the products' kernel time
is taken from the library's per-launch events, and the fastest variant is
stored in the library (tebd_tune_set) and in a JSON file, which later
processes load instead of timing again.  The variants agree to rounding
(the first two exactly); only speed depends on the choice.
"""
import json
import os

from . import _lib

ROW_BUCKETS = (128, 256, 512, 1024, 2048, 8192)
WIDTH_BUCKETS = (32, 64, 80, 128, 256)
VARIANTS = (0, 1, 2)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "tebd_rrsvd", "tuning.json")


def cache_path():
    return os.environ.get("TEBD_TUNE_CACHE", DEFAULT_CACHE)


def load(path=None):
    """Put the entries of a JSON cache into the library; returns them (or [])."""
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return []
    entries = data.get("entries", [])
    for e in entries:
        _lib.check(_lib.tebd_tune_set(e["precision"], e["rows"], e["width"], e["variant"]))
    return entries


def save(entries, path=None, device=""):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    with open(path, "w") as f:
        json.dump({"device": device, "entries": entries}, f, indent=1)
    return path


def _time_variant(torch, api, mats, k, p, variant, rows, width, reps):
    _lib.check(_lib.tebd_tune_set(0, rows, width, variant))
    api.rrsvd_truncate(mats, k, p, 2, 1e-10, 1504, 0)      # warm-up
    torch.cuda.synchronize()
    _lib.tebd_profile_enable(True)
    for r in range(reps):
        api.rrsvd_truncate(mats, k, p, 2, 1e-10, 1504, r + 1)
    torch.cuda.synchronize()
    prof = _lib.tebd_profile_read()
    _lib.tebd_profile_enable(False)
    return sum(v[0] for name, v in prof.items() if name.startswith("k_sketch")) / reps


def tune(buckets=((256, 64), (512, 80), (1024, 80), (2048, 80), (512, 128), (1024, 128),
                  (2048, 128), (4900, 256, 4)), batch=32, reps=3, path=None, seed=1504):
    """Time every variant for each (rows, width[, batch]) bucket; store and
    return the choices.  The batch of each bucket: `batch` (or the bucket's
    own count) square complex Gaussian matrices of the bucket's row count,
    sketch width = the bucket's width (k = width - 10, p = 10)."""
    import torch
    from . import api
    gen = torch.Generator(device="cuda")
    gen.manual_seed(int(seed))
    entries = []
    for bucket in buckets:
        rows, width = bucket[0], bucket[1]
        count = bucket[2] if len(bucket) > 2 else batch
        n = int(rows)
        mats = [torch.randn((n, n), dtype=torch.complex128, device="cuda", generator=gen)
                for _ in range(count)]
        k, p = max(1, int(width) - 10), 10
        ms = [_time_variant(torch, api, mats, k, p, v, rows, width, reps) for v in VARIANTS]
        best = VARIANTS[min(range(len(ms)), key=lambda i: ms[i])]
        _lib.check(_lib.tebd_tune_set(0, rows, width, best))
        entries.append({"precision": 0, "rows": int(rows), "width": int(width), "variant": best,
                        "sketch_ms": [round(x, 4) for x in ms]})
        del mats
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else ""
    save(entries, path, name)
    return entries


# TEBD sweeps read a table of their own (precision 2), bucketed by the MPS
# capacities (d_max chi_max rows, chi_max + p width), so that every rank mode
# takes the same variant.  A sweep batches a few large bond problems with
# many small ones: its sketch products are bound by the longest tile's chain
# of matrix-core steps, which a batch of equal synthetic matrices does not
# show, so these entries are tuned on the workload itself.
SWEEP_TABLE = 2


def tune_workload(run, workload, buckets, reps=2, path=None, precision=0):
    """Tune `buckets` of table `precision` on a real workload: `run()` executes
    it once (device work included).  Each variant is assigned to every bucket
    in turn and timed over `reps` runs after one warm-up; the fastest is kept
    for all of them, stored in the library and merged into the JSON cache
    (entries of other buckets are kept).  Returns the new entries."""
    import time
    import torch
    times = []
    for v in VARIANTS:
        for rows, width in buckets:
            _lib.check(_lib.tebd_tune_set(precision, rows, width, v))
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) / reps)
    best = VARIANTS[min(range(len(times)), key=lambda i: times[i])]
    entries = [{"precision": int(precision), "rows": int(r), "width": int(w), "variant": best,
                "workload": workload, "workload_s": [round(t, 5) for t in times]}
               for r, w in buckets]
    for e in entries:
        _lib.check(_lib.tebd_tune_set(precision, e["rows"], e["width"], best))
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {"device": "", "entries": []}
    keys = {(e["precision"], e["rows"], e["width"]) for e in entries}
    kept = [e for e in data.get("entries", []) if (e["precision"], e["rows"], e["width"]) not in keys]
    save(kept + entries, path, data.get("device", ""))
    return entries
