"""MI355X-native TEBD two-site update with reduced-rank randomized SVD.

Method: Tamascelli, Rosenbach, Plenio, arXiv:1504.00992.  The compute path is
the HIP library libtebd_rrsvd.so (C interface in include/tebd_rrsvd.h); this
package holds its ctypes binding (`_lib`), torch-facing wrappers (`api`) and
host-side gate builders (`models`).
"""
from . import _lib
from ._lib import (TebdError, TebdMps, TebdParams, load, params, tebd_last_error,
                   tebd_version)

__all__ = ["_lib", "TebdError", "TebdMps", "TebdParams", "load", "params", "tebd_last_error",
           "tebd_version"]
