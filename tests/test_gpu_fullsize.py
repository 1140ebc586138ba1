"""Parity at the benchmark's full sizes, in the launch designs the tuner picks
from (the fused 2D collide, the 3D ring collide, the ring-free tile collide):
D3Q19 256^3 and 384^3 and D2Q9 1024^2 droplets (radius L/4, Tr = 0.7, tanh
width 10) against the oracle on every node after a few steps, and mass conservation
over a longer run (a property at any size)."""
import numpy as np
import pytest

from paper_2205_09186_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-11


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_09186_amd import lbm
    lbm.lib()
    return lbm


def _workload(orc, lat, n, scheme):
    shape = (n, n, n) if lat == 1 else (n, n)
    g, l = orc.maxwell(0.7)
    rho0 = inputs.droplet(shape, 0.25 * n, 10.0, g, l)
    nz = n if lat == 1 else 1
    kw = dict(lattice=lat, nx=n, ny=n, nz=nz, tau=1.0, Tr=0.7, k=0.1, kappa=0.004, scheme=scheme)
    return shape, rho0, kw


def _design_variants(L, sim, lat, scheme):
    """One launch variant of each design the context offers: k_fused (CD
    schemes), the first ring variant, the tile collide with the two stencil
    marches and, where offered, with the one chemical-potential/force march,
    and every z-ring variant."""
    names = [sim.variant_name(v) for v in range(sim.num_variants)]
    out = []
    for kind in ("fused", "ring"):
        first = [v for v, n in enumerate(names) if n.startswith(kind)]
        out += first[:1]
    tiles = [v for v, n in enumerate(names) if n.startswith("tile") and " mf" not in n and " zr" not in n]
    mf = [v for v, n in enumerate(names) if n.endswith(" mf")]
    zr = [v for v, n in enumerate(names) if n.endswith(" zr")]     # the z-ring segments, every one offered
    out += tiles[-1:] + mf[:1] + zr
    return out


@pytest.mark.parametrize("lat,n,scheme,steps", [(1, 256, "CD6", 50), (1, 256, "OCFDS4", 2), (0, 1024, "CD6", 20),
                                                (0, 1024, "OCFDS4", 10), (1, 384, "CD6", 2), (1, 256, "E8", 2),
                                                (1, 256, "CD2", 5), (1, 256, "CD4", 5), (1, 384, "OCFDS4", 2)])
def test_full_size_against_oracle(L, orc, lat, n, scheme, steps):
    import torch
    shape, rho0, kw = _workload(orc, lat, n, L.SCHEMES[scheme])
    print(f"case full size lattice={lat} n={n} scheme={scheme} steps={steps}", flush=True)
    o = orc.Sim(orc.Params(**kw), rho0)
    o.step(steps)
    ro, vxo, vyo, vzo = o.macros()
    Uo, Mo = o.observables()
    del o
    d_rho0 = torch.from_numpy(rho0.reshape(-1)).cuda()
    probe = L.Simulation(L.Params(**kw), d_rho0)
    variants = _design_variants(L, probe, lat, L.SCHEMES[scheme])
    probe_names = [probe.variant_name(v) for v in range(probe.num_variants)]
    probe.close()
    del probe
    for v in variants:
        print(f"  variant {v} {probe_names[v]}", flush=True)
        sim = L.Simulation(L.Params(**kw), d_rho0)
        sim.set_variant(v)
        sim.step(steps)
        r, vx, vy, vz = sim.macros()
        d = max(np.abs(r - ro).max(), np.abs(vx - vxo).max(), np.abs(vy - vyo).max())
        if vz is not None:
            d = max(d, np.abs(vz - vzo).max())
        assert d <= TOL, (v, d)
        U, M, code = sim.spurious_max()
        assert code == 0
        assert U == pytest.approx(Uo, abs=TOL)
        assert M == pytest.approx(Mo, rel=1e-13)
        sim.close()
        del sim
        torch.cuda.empty_cache()


@pytest.mark.parametrize("lat,n", [(1, 256), (0, 1024)])
def test_full_size_mass_conservation(L, orc, lat, n):
    import torch
    shape, rho0, kw = _workload(orc, lat, n, L.CD6)
    sim = L.Simulation(L.Params(**kw), torch.from_numpy(rho0.reshape(-1)).cuda())
    sim.tune(steps=1)
    _, M0, _ = sim.spurious_max()
    sim.step(200)
    U, M, code = sim.spurious_max()
    assert code == 0 and np.isfinite(U)
    assert abs(M - M0) <= 1e-13 * M0
    sim.close()


def test_full_size_wall_against_oracle(L, orc):
    """The benchmark's wetting-boundary workload: D3Q19 256^3, an 8-plane solid
    floor under the droplet, mu_wall the Maxwell gas value k^2 psi'(rho_g),
    every tile variant against the oracle on every node after 2 steps."""
    import torch
    n, steps, k, Tr = 256, 2, 0.1, 0.7
    shape, rho0, kw = _workload(orc, 1, n, L.CD6)
    solid = np.zeros(shape, np.uint8)
    solid[:8] = 1
    g, _ = orc.maxwell(Tr)
    Tc, _, _ = orc.pr_critical()
    mu_wall = k * k * orc.pr_mub(g, Tr * Tc, orc.PR_A * orc.pr_alpha(Tr), orc.PR_B, orc.PR_R)
    print(f"case full size wall n={n} steps={steps}", flush=True)
    o = orc.Sim(orc.Params(solid=solid, mu_wall=mu_wall, **kw), rho0)
    o.step(steps)
    ro, vxo, vyo, vzo = o.macros()
    Uo, Mo = o.observables()
    del o
    d_rho0 = torch.from_numpy(rho0.reshape(-1)).cuda()
    probe = L.Simulation(L.Params(wall=1, mu_wall=mu_wall, **kw), d_rho0, solid=solid)
    nv = probe.num_variants
    names = [probe.variant_name(v) for v in range(nv)]
    probe.close()
    del probe
    assert names == ["tile 64x8 z32", "tile 64x16 z32", "tile 64x8 z64", "tile 64x16 z64"], names
    for v in range(nv):
        print(f"  variant {v}", flush=True)
        sim = L.Simulation(L.Params(wall=1, mu_wall=mu_wall, **kw), d_rho0, solid=solid)
        sim.set_variant(v)
        sim.step(steps)
        r, vx, vy, vz = sim.macros()
        d = max(np.abs(r - ro).max(), np.abs(vx - vxo).max(), np.abs(vy - vyo).max(), np.abs(vz - vzo).max())
        assert d <= TOL, (v, d)
        assert np.all(r[solid.astype(bool)] == 0.0)
        U, M, code = sim.spurious_max()
        assert code == 0 and U == pytest.approx(Uo, abs=TOL) and M == pytest.approx(Mo, rel=1e-13)
        sim.close()
