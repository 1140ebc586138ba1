"""GPU diagnostics (lbm_gradient, lbm_force) against the oracle's operators,
and the Sec 3.1-3.2 studies built on them."""
import numpy as np
import pytest

from paper_2205_09186_amd import inputs

pytestmark = pytest.mark.gpu
ALL = ["CD2", "CD4", "CD6", "E4", "E6", "E8", "E10", "OCFDS4", "CFDS4", "CFDS6", "CFDS8"]


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_09186_amd import lbm
    lbm.lib()
    return lbm


def _field(shape, seed):
    """A smooth periodic field with every axis varying (a few low modes)."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(s) * 2 * np.pi / s for s in shape], indexing="ij")
    f = np.full(shape, 2.0)
    for _ in range(4):
        k = [int(v) for v in rng.integers(1, 3, len(shape))]
        f += 0.3 * rng.standard_normal() * np.cos(sum(ki * g for ki, g in zip(k, grids)) + rng.uniform(0, 6))
    return f


@pytest.mark.parametrize("scheme", ALL)
@pytest.mark.parametrize("shape", [(37, 52), (9, 11, 14)])
def test_gradient_matches_oracle(L, orc, scheme, shape):
    if scheme == "E10" and len(shape) == 3:
        pytest.skip("E10 is two-dimensional only")
    f = _field(shape, 1)
    dim = len(shape)
    nz, ny, nx = ((1,) + shape) if dim == 2 else shape
    p = L.Params(lattice=0 if dim == 2 else 1, nx=nx, ny=ny, nz=nz, scheme=L.SCHEMES[scheme], Tr=0.9)
    sim = L.Simulation(p, np.full(shape, 3.0))
    g, lap = sim.gradient(f)
    go = np.zeros(3 * f.size)
    lo = np.zeros(f.size)
    lib = orc.lib()
    lib.orc_grad(dim, nx, ny, nz, L.SCHEMES[scheme], np.ascontiguousarray(f.reshape(-1)), go)
    lib.orc_lap(dim, nx, ny, nz, L.SCHEMES[scheme], np.ascontiguousarray(f.reshape(-1)), lo)
    scale = np.abs(go).max()
    np.testing.assert_allclose(g.cpu().numpy().reshape(dim, -1), go[: dim * f.size].reshape(dim, -1),
                               atol=1e-13 * scale)
    np.testing.assert_allclose(lap.cpu().numpy().reshape(-1), lo, atol=1e-13 * np.abs(lo).max())


@pytest.mark.parametrize("scheme", ALL)
@pytest.mark.parametrize("lat,shape", [(0, (45, 64)), (1, (12, 14, 16))])
def test_force_matches_oracle(L, orc, scheme, lat, shape):
    if scheme == "E10" and lat == 1:
        pytest.skip("E10 is two-dimensional only")
    g, l = orc.maxwell(0.8)
    rho0 = inputs.droplet(shape, min(shape) / 4, 4.0, g, l)
    nz, ny, nx = ((1,) + shape) if lat == 0 else shape
    kw = dict(lattice=lat, nx=nx, ny=ny, nz=nz, Tr=0.8, k=0.16, kappa=0.004, scheme=L.SCHEMES[scheme])
    sim = L.Simulation(L.Params(**kw), rho0)
    F, mu = sim.force()
    # the state the library holds is the density of feq(rho0, 0): rho0 itself
    Fo, muo = orc.force(orc.Params(**kw), rho0)
    assert np.abs(mu - muo).max() < 1e-13 * np.abs(muo).max()
    assert np.abs(F - Fo).max() < 1e-12 * np.abs(Fo).max()


def test_derivative_error_trends(L):
    """Fig 3(a): errors fall with k for a fixed scheme, and at large k the
    OCFDS4 error is below the explicit schemes' of the same or higher order."""
    from paper_2205_09186_amd import studies
    res = studies.derivative_errors(Tr=0.6, ks=(0.2, 0.8), kappa=0.04, n=192,
                                    schemes=("CD2", "CD4", "CD6", "OCFDS4"))
    lo, hi = res["0.2"]["errors"], res["0.8"]["errors"]
    for s in ("CD2", "CD4", "CD6", "OCFDS4"):
        assert lo[s] < hi[s], s
    assert hi["OCFDS4"] < hi["CD4"] and hi["OCFDS4"] < hi["CD2"]


def test_force_angle_trends(L):
    """Sec 3.2, Fig 6: the force of the Eq 26 droplet deviates least along the
    axes and diagonals; each step up in isotropy order lowers the deviation
    and raises the force error."""
    from paper_2205_09186_amd import studies
    iso = ("E4", "E6", "E8", "E10")
    res = studies.force_angles(n=160, r0=40.0, schemes=iso)
    for s in iso:
        b = res[s]["mean_abs_dtheta_deg_by_position_angle"]
        assert b["22.5"] > b["0"] and b["22.5"] > b["45"], (s, b)
    for a, b in zip(iso, iso[1:]):
        assert res[b]["rms_dtheta_deg"] < res[a]["rms_dtheta_deg"], (a, b)
        assert res[b]["rms_rel_force_error"] > res[a]["rms_rel_force_error"], (a, b)
