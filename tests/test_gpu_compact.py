"""The compact schemes' line solves on multi-segment lines: lines along x, y
and z longer than one 32-point segment, with a ragged last segment, solved in
one pass with exact periodic carries between segments (lines of up to 384
points, 12 segments), y and z lines of up to 1024 points by one wavefront
each (and, for comparison, by the chunked recursions), against the oracle's
Thomas + Sherman-Morrison solves."""
import numpy as np
import pytest

from paper_2205_09186_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_09186_amd import lbm
    lbm.lib()
    return lbm


@pytest.fixture(params=["segments", "waves", "chunks"])
def solver(request, monkeypatch):
    """Every line solver: the one-pass segment kernels (forced on these small
    grids), one wavefront per y or z line (exact scans across the lanes; the
    solver for y and z lines of 385 to 1024 points) and the chunked
    forward/backward recursions."""
    monkeypatch.setenv("LBM_SEG_MIN_LINES", "0" if request.param == "segments" else str(1 << 62))
    if request.param == "chunks":
        monkeypatch.setenv("LBM_NO_WAVE_LINES", "1")
    else:
        monkeypatch.delenv("LBM_NO_WAVE_LINES", raising=False)
    return request.param


@pytest.mark.parametrize("scheme", ["OCFDS4", "CFDS4", "CFDS6", "CFDS8"])
@pytest.mark.parametrize("shape", [(70, 37, 64), (33, 256, 20), (4, 65, 96), (300, 6, 8), (4, 1024, 6),
                                   (6, 4, 1000), (6, 384, 10), (384, 5, 12), (4, 333, 70), (4, 6, 350),
                                   (5, 4, 384)])
def test_gradient_multisegment_lines(L, orc, scheme, shape, solver):
    rng = np.random.default_rng(7)
    grids = np.meshgrid(*[np.arange(s) * 2 * np.pi / s for s in shape], indexing="ij")
    f = 2.0 + sum(0.2 * rng.standard_normal() * np.cos(sum(int(k) * g for k, g in zip(rng.integers(1, 4, 3), grids))
                                                        + rng.uniform(0, 6)) for _ in range(4))
    f += 1e-3 * rng.standard_normal(shape)      # every wavenumber present
    nz, ny, nx = shape
    p = L.Params(lattice=1, nx=nx, ny=ny, nz=nz, scheme=L.SCHEMES[scheme], Tr=0.9)
    sim = L.Simulation(p, np.full(shape, 3.0))
    g, lap = sim.gradient(f)
    go = np.zeros(3 * f.size)
    lo = np.zeros(f.size)
    lib = orc.lib()
    lib.orc_grad(3, nx, ny, nz, L.SCHEMES[scheme], np.ascontiguousarray(f.reshape(-1)), go)
    lib.orc_lap(3, nx, ny, nz, L.SCHEMES[scheme], np.ascontiguousarray(f.reshape(-1)), lo)
    scale = np.abs(go).max()
    np.testing.assert_allclose(g.cpu().numpy().reshape(3, -1), go.reshape(3, -1), atol=1e-13 * scale)
    np.testing.assert_allclose(lap.cpu().numpy().reshape(-1), lo, atol=1e-13 * np.abs(lo).max())


@pytest.mark.parametrize("scheme", ["OCFDS4", "CFDS8"])
@pytest.mark.parametrize("shape", [(70, 37, 64), (600, 40), (370, 40)])
def test_step_multisegment_lines(L, orc, scheme, shape, solver):
    g, l = orc.maxwell(0.9)
    rho0 = inputs.droplet(shape, 12, 4.0, g, l)
    nz, ny, nx = shape if len(shape) == 3 else (1,) + shape
    kw = dict(lattice=len(shape) - 2, nx=nx, ny=ny, nz=nz, Tr=0.9, k=0.16, kappa=0.004, scheme=L.SCHEMES[scheme])
    print(f"case compact step shape={shape} scheme={scheme}", flush=True)
    sim = L.Simulation(L.Params(**kw), rho0)
    sim.step(30)
    o = orc.Sim(orc.Params(**kw), rho0)
    o.step(30)
    r, vx, vy, vz = sim.macros()
    ro, vxo, vyo, vzo = o.macros()
    pairs = [(r, ro), (vx, vxo), (vy, vyo)] + ([(vz, vzo)] if vz is not None else [])
    d = max(np.abs(a - b).max() for a, b in pairs)
    assert d <= 1e-11, d


@pytest.mark.parametrize("lat,shape,scheme", [(0, (96, 130), "OCFDS4"), (1, (20, 24, 28), "CFDS6")])
def test_concurrent_axes_equal_sequential(L, orc, lat, shape, scheme, monkeypatch):
    """The per-axis derivative passes on branch streams (forked and joined by
    events, also inside the captured step graph) give bitwise the state of the
    same passes run one after another."""
    g, l = orc.maxwell(0.8)
    rho0 = inputs.droplet(shape, min(shape) / 4, 4.0, g, l)
    nz, ny, nx = ((1,) + shape) if lat == 0 else shape
    p = L.Params(lattice=lat, nx=nx, ny=ny, nz=nz, Tr=0.8, scheme=L.SCHEMES[scheme])
    a = L.Simulation(p, rho0)
    monkeypatch.setenv("LBM_NO_CONC", "1")
    b = L.Simulation(p, rho0)
    monkeypatch.delenv("LBM_NO_CONC")
    for n in (1, 8, 3):        # plain launches and graph replays
        a.step(n)
        b.step(n)
    assert np.array_equal(a.populations(), b.populations())
    Fa, mua = a.force()
    Fb, mub = b.force()
    assert np.array_equal(Fa, Fb) and np.array_equal(mua, mub)
