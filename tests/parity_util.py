"""Comparison helpers shared by the GPU parity tests."""
import numpy as np


def relinf(a, b):
    """max |a - b| / max |b| (relative infinity-norm distance)."""
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def fp32_cycle_bound(Oc, r):
    """(binary32 oracle cycle, binary64 oracle cycle, bound) for one V-cycle
    applied to r.  The GPU and the oracle round the same binary32 operations in
    different orders, so each lies about delta from the binary64 cycle, delta
    being the oracle's own binary32-versus-binary64 distance on r (about
    1e-7 .. 7e-7 on the test workloads).  The bound is 8 delta."""
    z32 = Oc.vcycle32(r.astype(np.float32)).astype(np.float64)
    z64 = Oc.vcycle(r)
    return z32, z64, 8.0 * relinf(z32, z64)
