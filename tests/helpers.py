"""Shared test helpers (no method arithmetic here)."""
import ctypes

import numpy as np

from paper_2606_02169_amd import _lib as L


def host_plan(model, require_hermitian=True):
    """Create a plan through the raw C ABI (host only; no GPU needed).  Returns (status, handle)."""
    from paper_2606_02169_amd.plan import _local_array, _site_array, _term_array
    h = ctypes.c_void_p()
    ops = getattr(model, "local_ops", ())
    la, keep = _local_array(ops)
    st = L.lib().mrmf_plan_create_ex(len(model.sites), _site_array(model.sites), len(model.terms),
                                     _term_array(model.terms), model.n_params,
                                     L.MRMF_REQUIRE_HERMITIAN if require_hermitian else 0, len(ops), la,
                                     ctypes.byref(h))
    del keep
    return st, h


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)
