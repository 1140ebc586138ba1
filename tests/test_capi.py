"""CPU-side checks of the C ABI library: it loads, exports every symbol the
header declares, validates parameters before touching the GPU, and its host
EOS helpers agree with the oracle."""
import ctypes as C
import os
import re

import pytest

from paper_2205_09186_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:lbm|mlp)_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = lbm.lib()
    names = header_symbols()
    assert "lbm_init" in names and "lbm_step" in names and "lbm_macros" in names and "lbm_spurious_max" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lbm.SYMBOLS)


def test_workspace_validation():
    ok = lbm.Params(lattice=lbm.D3Q19, nx=16, ny=16, nz=16, scheme=lbm.CD6)
    nb = lbm.workspace_bytes(ok)
    assert nb >= 2 * 19 * 16 ** 3 * 8
    bad = [dict(tau=0.5), dict(Tr=1.0), dict(Tr=0.0), dict(k=0.0), dict(kappa=-1.0), dict(scheme=11),
           dict(scheme=-1), dict(scheme=lbm.E10),
           dict(nz=1), dict(nx=3), dict(lattice=2), dict(collision=2), dict(collision=lbm.MRT),
           dict(collision=lbm.MRT, s_e=2.0), dict(s_q=-1.0)]
    for b in bad:
        q = lbm.Params(**{**ok.__dict__, **b})
        assert lbm.workspace_bytes(q) == 0, b
    q2 = lbm.Params(lattice=lbm.D2Q9, nx=16, ny=16, nz=2)
    assert lbm.workspace_bytes(q2) == 0
    # E6 in both dimensions, E10 in 2D only
    assert lbm.workspace_bytes(lbm.Params(**{**ok.__dict__, "scheme": lbm.E6})) > 0
    assert lbm.workspace_bytes(lbm.Params(lattice=lbm.D2Q9, nx=16, ny=16, scheme=lbm.E10)) > 0
    # MRT is defined for D2Q9 (Eq 3)
    assert lbm.workspace_bytes(lbm.Params(lattice=lbm.D2Q9, nx=16, ny=16, collision=lbm.MRT)) > 0
    # compact schemes need the gradient fields as well
    assert lbm.workspace_bytes(lbm.Params(**{**ok.__dict__, "scheme": lbm.OCFDS4})) > nb


def test_init_rejects_bad_arguments_without_gpu():
    L = lbm.lib()
    p = lbm.Params(lattice=lbm.D2Q9, nx=8, ny=8).c()
    ctx = C.c_void_p()
    rc = L.lbm_init(C.byref(p), None, 0, None, 0, None, C.byref(ctx))
    assert rc == lbm.LBM_EINVAL and ctx.value is None
    assert "rho0" in L.lbm_last_error(None).decode()
    bad = lbm.Params(lattice=lbm.D2Q9, nx=8, ny=8, tau=0.4).c()
    rc = L.lbm_init(C.byref(bad), None, 0, None, 0, None, C.byref(ctx))
    assert rc == lbm.LBM_EINVAL and "tau" in L.lbm_last_error(None).decode()
    # workspace too small is reported before any device work
    import numpy as np
    rho = np.ones(64)
    buf = (C.c_ubyte * 4096)()
    addr = (C.addressof(buf) + 255) // 256 * 256
    rc = L.lbm_init(C.byref(p), rho.ctypes.data_as(C.c_void_p), 0, C.c_void_p(addr), 1024, None, C.byref(ctx))
    assert rc == lbm.LBM_ENOSPC
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_last_error(None) is not None
    L.lbm_free(None)
    # walls: lbm_init refuses wall = 1, lbm_init_wall needs it and a mask
    pw = lbm.Params(lattice=lbm.D2Q9, nx=8, ny=8, wall=1).c()
    rc = L.lbm_init(C.byref(pw), rho.ctypes.data_as(C.c_void_p), 0, C.c_void_p(addr), 4000, None, C.byref(ctx))
    assert rc == lbm.LBM_EINVAL and "lbm_init_wall" in L.lbm_last_error(None).decode()
    mask = np.zeros(64, np.uint8)
    rc = L.lbm_init_wall(C.byref(p), rho.ctypes.data_as(C.c_void_p), mask.ctypes.data_as(C.c_void_p), 0,
                         C.c_void_p(addr), 4000, None, C.byref(ctx))
    assert rc == lbm.LBM_EINVAL and "wall = 1" in L.lbm_last_error(None).decode()
    rc = L.lbm_init_wall(C.byref(pw), rho.ctypes.data_as(C.c_void_p), None, 0, C.c_void_p(addr), 4000, None,
                         C.byref(ctx))
    assert rc == lbm.LBM_EINVAL and "solid" in L.lbm_last_error(None).decode()


def test_wall_parameters_are_validated():
    base = dict(lattice=lbm.D2Q9, nx=16, ny=16, wall=1, scheme=lbm.CD6, mu_wall=0.01)
    ok = lbm.workspace_bytes(lbm.Params(**base))
    # the layer map (1 byte per node) and the bounce-back mask (4 bytes per node),
    # each 256-byte aligned
    assert ok == lbm.workspace_bytes(lbm.Params(**{**base, "wall": 0})) + 256 + 1024
    for bad in (dict(scheme=lbm.E4), dict(scheme=lbm.OCFDS4), dict(scheme=lbm.CFDS6), dict(wall=2),
                dict(mu_wall=float("nan"))):
        assert lbm.workspace_bytes(lbm.Params(**{**base, **bad})) == 0, bad


def test_critical_point_matches_oracle(orc):
    Tc, rc, pc = lbm.critical()
    To, ro, po = orc.pr_critical()
    assert Tc == pytest.approx(To, rel=1e-12)
    assert rc == pytest.approx(ro, rel=1e-10)
    assert pc == pytest.approx(po, rel=1e-12)


@pytest.mark.parametrize("Tr", [0.95, 0.8, 0.7, 0.6, 0.4, 0.3, 0.2])
def test_coexistence_matches_oracle(orc, Tr):
    g, l = lbm.coexistence(Tr)
    go, lo = orc.maxwell(Tr)
    assert g == pytest.approx(go, rel=1e-11)
    assert l == pytest.approx(lo, rel=1e-13)
    with pytest.raises(lbm.LbmError):
        lbm.coexistence(1.2)


def test_probe_copy_validates_before_any_launch():
    """The copy probe rejects a bad lattice, size or pointer with LBM_EINVAL
    (these checks run before any device work)."""
    L = lbm.lib()
    one = C.c_void_p(8)   # never dereferenced: every call below fails validation
    bad = [(2, 4, 4, 4, one, one), (lbm.D3Q19, 0, 4, 4, one, one), (lbm.D2Q9, 4, 4, 2, one, one),
           (lbm.D3Q19, 4, 4, 4, None, one), (lbm.D3Q19, 4, 4, 4, one, None), (lbm.D3Q19, 8192, 8192, 8192, one, one)]
    for lat, nx, ny, nz, s, d in bad:
        assert L.lbm_probe_copy(lat, nx, ny, nz, s, d, 0, None) == lbm.LBM_EINVAL


def test_static_sum_rejects_bad_arguments_without_gpu():
    """lbm_sum_static refuses a size beyond its fixed scratch, an empty input
    and NULL pointers before it touches a device."""
    L = lbm.lib()
    nmax = L.lbm_sum_static_max()
    assert nmax == 1 << 26
    out = C.c_double(-1.0)
    fake = C.c_void_p(4096)   # never dereferenced: every case fails validation first
    assert L.lbm_sum_static(fake, nmax + 1, C.byref(out), None) == lbm.LBM_EINVAL
    assert "exceeds the maximum" in L.lbm_last_error(None).decode()
    assert L.lbm_sum_static(fake, 0, C.byref(out), None) == lbm.LBM_EINVAL
    assert L.lbm_sum_static(None, 10, C.byref(out), None) == lbm.LBM_EINVAL
    assert L.lbm_sum_static(fake, 10, None, None) == lbm.LBM_EINVAL
    assert out.value == -1.0


def test_degenerate_sizes_are_refused_without_gpu():
    """Grids below the smallest periodic lattice (nx or ny < 4, nz < 4 in 3D,
    nz != 1 in 2D) and an empty batch are refused before any device work."""
    L = lbm.lib()
    for kw in (dict(lattice=lbm.D2Q9, nx=3, ny=8), dict(lattice=lbm.D2Q9, nx=8, ny=0),
               dict(lattice=lbm.D2Q9, nx=8, ny=8, nz=2), dict(lattice=lbm.D3Q19, nx=8, ny=8, nz=3)):
        p = lbm.Params(**kw).c()
        assert L.lbm_workspace_bytes(C.byref(p)) == 0, kw
    p = lbm.Params(lattice=lbm.D2Q9, nx=8, ny=8).c()
    assert L.lbm_batch_workspace_bytes(C.byref(p), 0) == 0
    out = C.c_void_p()
    rc = L.lbm_batch_init(C.byref(p), None, 0, None, 0, None, C.byref(out))
    assert rc == lbm.LBM_EINVAL and out.value is None
