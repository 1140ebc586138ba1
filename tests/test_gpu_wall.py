"""GPU <-> oracle parity of the step with the chemical-potential wetting
boundary (Appendix, Eq A.1; halfway bounce-back), through lbm_init_wall.
Every comparison runs both sides on the same seeded density and solid mask;
fluid nodes must agree to 1e-11 in rho and v, solid nodes report zeros."""
import numpy as np
import pytest

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


def _mu_M(orc, Tr, k):
    g, _ = orc.maxwell(Tr)
    Tc, _, _ = orc.pr_critical()
    return k * k * orc.pr_mub(g, Tr * Tc, orc.PR_A * orc.pr_alpha(Tr), orc.PR_B, orc.PR_R)


def _case(orc, lat, shape, floor, ball, seed=0, Tr=0.8):
    """A solid floor `floor` nodes thick (plus, if ball, a solid sphere in the
    fluid) and a droplet resting above the floor; all from a seeded rng."""
    rng = np.random.default_rng(seed)
    idx = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    solid = np.zeros(shape, np.uint8)
    solid[:floor] = 1
    g, l = orc.maxwell(Tr)
    c = [floor + shape[0] * 0.3] + [s / 2 + 0.37 for s in shape[1:]]
    r = np.sqrt(sum((i - ci) ** 2 for i, ci in zip(idx, c)))
    R = 0.22 * min(shape)
    rho0 = (l + g) / 2 - (l - g) / 2 * np.tanh(2 * (r - R) / 4.0)
    rho0 *= 1 + 1e-6 * rng.uniform(-1, 1, shape)
    if ball:
        cb = [shape[0] * 0.75] + [s * 0.3 for s in shape[1:]]
        solid[np.sqrt(sum((i - ci) ** 2 for i, ci in zip(idx, cb))) < 0.12 * min(shape)] = 1
    return solid, rho0


def _pair(L, orc, lat, shape, scheme, steps, solid, rho0, mu_rel, Tr=0.8, k=0.16, kappa=0.004, tau=1.0,
          collision=0, s_e=0.0):
    nz, ny, nx = ((1,) + tuple(shape)) if lat == 0 else tuple(shape)
    mu_wall = _mu_M(orc, Tr, k) * (1.0 + mu_rel)
    kw = dict(lattice=lat, nx=nx, ny=ny, nz=nz, tau=tau, Tr=Tr, k=k, kappa=kappa, scheme=scheme,
              collision=collision, s_e=s_e, mu_wall=mu_wall)
    print(f"case lattice={lat} shape={shape} scheme={scheme} steps={steps} mu_rel={mu_rel}", flush=True)
    sim = L.Simulation(L.Params(wall=1, **kw), rho0, solid=solid)
    sim.step(steps)
    o = orc.Sim(orc.Params(solid=solid, **kw), rho0)
    o.step(steps)
    return sim, o


def _compare(sim, o, solid):
    r, vx, vy, vz = sim.macros()
    ro, vxo, vyo, vzo = o.macros()
    assert np.all(np.isfinite(ro)), "oracle diverged"
    d = {"rho": np.abs(r - ro).max(), "vx": np.abs(vx - vxo).max(), "vy": np.abs(vy - vyo).max()}
    if vz is not None:
        d["vz"] = np.abs(vz - vzo).max()
    assert max(d.values()) <= TOL, d
    s = solid.astype(bool)
    assert np.all(r[s] == 0.0) and np.all(vx[s] == 0.0)
    U, M, code = sim.spurious_max()
    Uo, Mo = o.observables()
    assert code == 0
    assert U == pytest.approx(Uo, abs=TOL)
    assert M == pytest.approx(Mo, rel=1e-13)
    return d


@pytest.mark.parametrize("scheme,Tr,mu_rel", [("CD2", 0.9, 0.0), ("CD4", 0.8, 2.0), ("CD6", 0.8, -2.0),
                                             ("CD6", 0.8, 5.0)])
def test_wall_2d_droplet(L, orc, scheme, Tr, mu_rel):
    solid, rho0 = _case(orc, 0, (53, 70), 5, ball=True, Tr=Tr)
    sim, o = _pair(L, orc, 0, (53, 70), L.SCHEMES[scheme], 400, solid, rho0, mu_rel, Tr=Tr)
    _compare(sim, o, solid)


@pytest.mark.parametrize("scheme", ["CD4", "CD6"])
def test_wall_3d_droplet(L, orc, scheme):
    solid, rho0 = _case(orc, 1, (22, 20, 18), 4, ball=True)
    sim, o = _pair(L, orc, 1, (22, 20, 18), L.SCHEMES[scheme], 80, solid, rho0, 1.0)
    _compare(sim, o, solid)


@pytest.mark.parametrize("lat,tau,collision", [(0, 0.8, 0), (1, 1.3, 0), (0, 0.9, 1)])
def test_wall_relaxation_and_mrt(L, orc, lat, tau, collision):
    shape = (40, 45) if lat == 0 else (16, 18, 14)
    solid, rho0 = _case(orc, lat, shape, 4, ball=False, seed=3)
    sim, o = _pair(L, orc, lat, shape, L.CD4, 150, solid, rho0, 1.0, tau=tau, collision=collision,
                   s_e=1.25 if collision else 0.0)
    _compare(sim, o, solid)


def test_wall_thin_solid_and_periodic_images(L, orc):
    """A solid slab only two nodes thick with CD6 (three layers wanted): both
    rows are layer 1, one from each face, and the stencils of the fluid on
    either side reach through the slab.  Such a slab is thinner than the
    scheme's reach and the run diverges after ~60 steps (oracle and GPU
    alike), so the comparison stops at 30."""
    shape = (30, 41)
    solid = np.zeros(shape, np.uint8)
    solid[10:12] = 1
    g, l = orc.maxwell(0.8)
    yy, xx = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    rho0 = (l + g) / 2 - (l - g) / 2 * np.tanh(2 * (np.hypot(xx - 20.3, yy - 21.5) - 5.0) / 4.0)
    sim, o = _pair(L, orc, 0, shape, L.CD6, 30, solid, rho0, 0.5)
    _compare(sim, o, solid)


def test_wall_force_and_populations(L, orc):
    import torch
    solid, rho0 = _case(orc, 0, (33, 40), 4, ball=True, seed=5)
    mu_wall = _mu_M(orc, 0.8, 0.16) * 3.0
    kw = dict(lattice=0, nx=40, ny=33, Tr=0.8, k=0.16, kappa=0.004, scheme=L.CD6, mu_wall=mu_wall)
    sim = L.Simulation(L.Params(wall=1, **kw), rho0, solid=solid)
    F, mu = sim.force()
    Fo, muo = orc.force(orc.Params(solid=solid, **kw), rho0)
    fluid = solid == 0
    assert np.abs(mu[fluid] - muo[fluid]).max() < 1e-13 * np.abs(muo).max()
    assert np.all(mu[~fluid] == mu_wall) and np.all(muo[~fluid] == mu_wall)
    assert np.abs(F - Fo).max() < 1e-12 * np.abs(Fo).max()
    assert np.all(F[:, ~fluid] == 0.0)
    # the state after some steps, as populations
    sim.step(30)
    o = orc.Sim(orc.Params(solid=solid, **kw), rho0)
    o.step(30)
    fa, fo = sim.populations(), o.populations()
    assert np.abs(fa - fo).max() < 1e-12
    assert np.all(fa[:, ~fluid.reshape(-1)] == 0.0)
    # device-side inputs give the same state
    dev = L.Simulation(L.Params(wall=1, **kw), torch.from_numpy(rho0.reshape(-1)).cuda(),
                       solid=torch.from_numpy(solid.reshape(-1)).cuda())
    dev.step(30)
    assert np.array_equal(dev.populations(), fa)


def test_wall_fixed_point_uniform_fluid(L, orc):
    """A uniform fluid at rest around a solid ball, with the wall's chemical
    potential equal to the fluid's, stays put."""
    shape = (24, 26, 20)
    idx = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    solid = (np.sqrt(sum((i - s / 2) ** 2 for i, s in zip(idx, shape))) < 6).astype(np.uint8)
    rho_u, Tr, k = 3.1, 0.8, 0.16
    Tc, _, _ = orc.pr_critical()
    mu_w = k * k * orc.pr_mub(rho_u, Tr * Tc, orc.PR_A * orc.pr_alpha(Tr), orc.PR_B, orc.PR_R)
    p = L.Params(lattice=1, nx=20, ny=26, nz=24, Tr=Tr, k=k, scheme=L.CD6, wall=1, mu_wall=mu_w, tau=0.8)
    sim = L.Simulation(p, np.full(shape, rho_u), solid=solid)
    f0 = sim.populations()
    sim.step(20)
    assert np.abs(sim.populations() - f0).max() < 1e-14


@pytest.mark.parametrize("lat,shape,scheme,mu_rel,coll", [(0, (48, 128), "CD6", 2.0, 0), (0, (64, 64), "CD4", -1.0, 1),
                                                         (1, (24, 16, 64), "CD4", 1.0, 0),
                                                         (1, (20, 32, 64), "CD6", 3.0, 0)])
def test_wall_tile_collide(L, orc, lat, shape, scheme, mu_rel, coll, monkeypatch):
    """Grids tiled by 64 x 8 take the tile collide with bounce-back (every tile
    height and z-segment length) against the oracle and against the
    node-parallel path."""
    solid, rho0 = _case(orc, lat, shape, 5 if lat == 0 else 4, ball=True, seed=2)
    nz, ny, nx = ((1,) + tuple(shape)) if lat == 0 else tuple(shape)
    kw = dict(lattice=lat, nx=nx, ny=ny, nz=nz, tau=1.0 if not coll else 0.9, Tr=0.8, k=0.16, kappa=0.004,
              scheme=L.SCHEMES[scheme], collision=coll, s_e=1.25 if coll else 0.0,
              mu_wall=_mu_M(orc, 0.8, 0.16) * (1.0 + mu_rel))
    steps = 120 if lat == 0 else 40
    print(f"case wall tile lattice={lat} shape={shape} scheme={scheme}", flush=True)
    monkeypatch.setenv("LBM_NO_FUSED", "1")
    ref = L.Simulation(L.Params(wall=1, **kw), rho0, solid=solid)
    monkeypatch.delenv("LBM_NO_FUSED")
    ref.step(steps)
    o = orc.Sim(orc.Params(solid=solid, **kw), rho0)
    o.step(steps)
    probe = L.Simulation(L.Params(wall=1, **kw), rho0, solid=solid)
    nv = probe.num_variants
    # tile heights 8 and 16; in 3D z segments of 32 and 64 planes
    assert nv == (2 if ny % 16 == 0 else 1) * (2 if lat == 1 else 1)
    assert [n for n, _ in probe.step_timed(1)][-2:] == ["k_tile", "k_fix"]
    for v in range(nv):
        sim = L.Simulation(L.Params(wall=1, **kw), rho0, solid=solid)
        sim.set_variant(v)
        sim.step(steps)
        assert np.abs(sim.populations() - ref.populations()).max() < 1e-13, v
        _compare(sim, o, solid)
