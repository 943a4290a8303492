"""The allocation-free FP64 dot product (rt_dot_noalloc, partials in the
library's static device array) against rt_dot, through the C ABI: two calls
in a row, the second on a smaller input (stale partials of the first call
stay in the array and must not be read), bitwise equal to rt_dot and within
1e-12 of numpy's FP64 sum."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1809_09725_amd import inputs, rt4d

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def dot(fn, x, y):
    out = ctypes.c_double()
    rc = fn(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.numel(),
            ctypes.byref(out), ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream))
    assert rc == rt4d.RT_OK, rt4d.lib().rt_last_error().decode()
    return out.value


def test_noalloc_dot_equals_dot_two_calls_second_smaller():
    torch.cuda.set_device(DEV)
    L = rt4d.lib()
    for n, seed in ((3_000_001, 1), (777, 2), (0, 3)):
        xh = inputs.uniform((n,), seed)
        yh = inputs.uniform((n,), seed + 10)
        x = torch.from_numpy(xh).to(DEV)
        y = torch.from_numpy(yh).to(DEV)
        a = dot(L.rt_dot_noalloc, x, y)
        b = dot(L.rt_dot, x, y)
        want = float(np.dot(xh.astype(np.float64), yh.astype(np.float64)))
        print(f"n={n}: noalloc {a!r} dot {b!r} numpy {want!r}", flush=True)
        assert a == b
        assert abs(a - want) <= 1e-12 * max(1.0, float(np.sum(np.abs(xh.astype(np.float64) * yh))))
        sq = dot(L.rt_dot_noalloc, x, x)
        assert sq == dot(L.rt_dot, x, x)


def test_noalloc_dot_rejects_null():
    out = ctypes.c_double()
    rc = rt4d.lib().rt_dot_noalloc(None, None, 5, ctypes.byref(out), None)
    assert rc == rt4d.RT_E_ARG
