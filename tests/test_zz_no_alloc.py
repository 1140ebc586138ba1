"""The allocation-free sum (lbm_sum_static) against lbm_sum, through the C ABI.

Both run the same kernels in the same order, so the results must agree bit for
bit; two calls in a row, the second on a smaller input, show that the shared
static scratch keeps no state that leaks into the next call."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_2205_09186_amd import inputs, lbm

pytestmark = pytest.mark.gpu


def _sum_with_scratch(L, x, n, stream):
    import torch
    scratch = torch.empty(max(1, L.lbm_sum_scratch_bytes(n) // 8), dtype=torch.float64, device=x.device)
    out = C.c_double()
    rc = L.lbm_sum(C.c_void_p(x.data_ptr()), n, C.c_void_p(scratch.data_ptr()), C.byref(out), stream)
    assert rc == lbm.LBM_OK, L.lbm_last_error(None)
    return out.value


def _sum_static(L, x, n, stream):
    out = C.c_double()
    rc = L.lbm_sum_static(C.c_void_p(x.data_ptr()), n, C.byref(out), stream)
    assert rc == lbm.LBM_OK, L.lbm_last_error(None)
    return out.value


@pytest.mark.parametrize("use_torch_stream", [False, True])
def test_static_sum_matches_lbm_sum_twice(use_torch_stream):
    import torch
    L = lbm.lib()
    nmax = L.lbm_sum_static_max()
    assert nmax == 1 << 26
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream) if use_torch_stream else None
    # first a large ragged input, then a much smaller one
    for n in (12_345_679, 1_037):
        h = 1.0 + inputs.noise((n,), amplitude=0.5, instance_id=n)
        x = torch.from_numpy(h).cuda()
        print(f"lbm_sum_static n={n} torch_stream={use_torch_stream}", flush=True)
        a = _sum_static(L, x, n, stream)
        b = _sum_with_scratch(L, x, n, stream)
        assert a == b, (n, a, b)
        exact = math.fsum(h.tolist())
        assert abs(a - exact) <= 1e-13 * abs(exact), (n, a, exact)


def test_static_sum_at_its_maximum_then_small():
    import torch
    L = lbm.lib()
    n = int(L.lbm_sum_static_max())
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    x[::7] = 0.5
    print(f"lbm_sum_static n={n} (maximum)", flush=True)
    a = _sum_static(L, x, n, None)
    assert a == _sum_with_scratch(L, x, n, None)
    assert a == n - 0.5 * ((n + 6) // 7)
    y = torch.arange(1, 301, dtype=torch.float64, device="cuda")
    assert _sum_static(L, y, 300, None) == 45150.0
    # one past the maximum is refused before any launch
    out = C.c_double(-1.0)
    assert L.lbm_sum_static(C.c_void_p(x.data_ptr()), n + 1, C.byref(out), None) == lbm.LBM_EINVAL
    assert out.value == -1.0
    assert "exceeds the maximum" in L.lbm_last_error(None).decode()
