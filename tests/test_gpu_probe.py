"""The copy probe that measures the memory ceiling of the step's access
pattern: the aligned copy reproduces every population array, and the pull
moves array i by one lattice velocity e_i (dst_i(x) = src_i(x - e_i),
periodic), the velocities over all arrays being the lattice's set."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_09186_amd import lbm
    lbm.lib()
    return lbm


@pytest.mark.parametrize("lat,shape", [(1, (6, 5, 7)), (0, (1, 9, 11))])
def test_probe_copy_aligned_and_pull(L, orc, lat, shape):
    import torch
    nz, ny, nx = shape
    n = nx * ny * nz
    e, _ = orc.lattice(lat)
    q = len(e)
    src = torch.rand(q * n, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    stream = torch.cuda.current_stream()
    for pull in (0, 1):
        dst.zero_()
        assert L.lib().lbm_probe_copy(lat, nx, ny, nz, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                      pull, C.c_void_p(stream.cuda_stream)) == L.LBM_OK
        torch.cuda.synchronize()
        s = src.cpu().numpy().reshape(q, nz, ny, nx)
        d = dst.cpu().numpy().reshape(q, nz, ny, nx)
        if not pull:
            assert np.array_equal(s, d)
            continue
        used = []
        for i in range(q):
            hits = [tuple(v) for v in e if np.array_equal(d[i], np.roll(s[i], (v[2], v[1], v[0]), axis=(0, 1, 2)))]
            assert hits, i
            used.append(hits[0])
        assert sorted(used) == sorted(tuple(v) for v in e)
