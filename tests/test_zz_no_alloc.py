"""GPU: the allocation-free inference entry point against ugks_mlp_forward.

ugks_mlp_forward_noalloc runs the same bf16 matrix-core inference with its
staging rows in a static device array instead of allocated buffers.  Called
through the C ABI twice in a row, the second time with fewer rows (the array
keeps the first call's contents), it must give the outputs of
ugks_mlp_forward on the same device rows, bit for bit (same kernel, same
inputs); sizes beyond the array's capacity are refused before any work.

The test's own device buffers come from the HIP runtime the library is
linked against (by its soname, once the library is loaded), so the test
does not depend on which other GPU users the process has loaded first.
"""

import ctypes as C

import numpy as np
import pytest

from paper_2606_15720_amd import ugks as U
from paper_2606_15720_amd import warmstart as WS

pytestmark = pytest.mark.gpu

H2D, D2H = 1, 2  # hipMemcpyHostToDevice, hipMemcpyDeviceToHost


def _hip():
    U.load_library()
    hip = C.CDLL("libamdhip64.so.7")  # already loaded as the library's dependency
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipFree.argtypes = [C.c_void_p]
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipSetDevice.argtypes = [C.c_int]
    for f in (hip.hipMalloc, hip.hipFree, hip.hipMemcpy, hip.hipSetDevice, hip.hipDeviceSynchronize):
        f.restype = C.c_int
    return hip


class _DevRows:
    """rows x 9 floats of device memory (test-side buffer)."""

    def __init__(self, hip, rows):
        self.hip, self.n = hip, rows * 9 * 4
        self.p = C.c_void_p()
        assert hip.hipMalloc(C.byref(self.p), self.n) == 0

    def put(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        assert a.nbytes == self.n
        assert self.hip.hipMemcpy(self.p, a.ctypes.data_as(C.c_void_p), self.n, H2D) == 0

    def get(self):
        out = np.empty(self.n // 4, dtype=np.float32)
        assert self.hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), self.p, self.n, D2H) == 0
        return out.reshape(-1, 9)

    def free(self):
        self.hip.hipFree(self.p)


def _net():
    rng = np.random.default_rng(17)
    p = (WS.init_params(3) + rng.normal(0, 0.05, WS.NPARAM)).astype(np.float32)
    si = rng.uniform(0.5, 2.0, 9).astype(np.float32)
    so = rng.uniform(0.5, 2.0, 9).astype(np.float32)
    return U.MLP(p, si, so)


def test_noalloc_inference_matches_the_allocating_entry_point():
    hip = _hip()
    assert hip.hipSetDevice(0) == 0
    net = _net()
    rng = np.random.default_rng(5)
    for rows in (3001, 517):  # not multiples of the 16-row tile; the second call is smaller
        x = rng.normal(0.0, 0.7, (rows, 9)).astype(np.float32)
        xd, yref, ynew = _DevRows(hip, rows), _DevRows(hip, rows), _DevRows(hip, rows)
        xd.put(x)
        ynew.put(np.full((rows, 9), np.nan, dtype=np.float32))
        print(f"rows {rows}: ugks_mlp_forward", flush=True)
        net.forward_device(xd.p.value, rows, yref.p.value)
        print(f"rows {rows}: ugks_mlp_forward_noalloc", flush=True)
        net.forward_noalloc(xd.p.value, rows, ynew.p.value)
        assert hip.hipDeviceSynchronize() == 0
        a, b = yref.get(), ynew.get()
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b), np.abs(a - b).max()
        # and the host-buffer path of the allocating entry point
        assert np.array_equal(net.forward(x), b)
        for d in (xd, yref, ynew):
            d.free()
    net.close()


def test_noalloc_inference_refuses_sizes_beyond_its_array():
    hip = _hip()
    assert hip.hipSetDevice(0) == 0
    net = _net()
    x = _DevRows(hip, 4)
    with pytest.raises(U.UGKSError) as e:
        net.forward_noalloc(x.p.value, U.NOALLOC_MAX_ROWS + 1, x.p.value)
    assert e.value.code == U.UGKS_EINVAL and "allocation-free" in str(e.value)
    with pytest.raises(U.UGKSError):
        net.forward_noalloc(x.p.value, -1, x.p.value)
    net.forward_noalloc(x.p.value, 0, x.p.value)  # nothing to do
    x.free()
    net.close()
