"""Pins of the oracle's wetting boundary (Appendix, Eq A.1) against what the
definition and the mathematics fix: an all-fluid mask is the periodic step;
on a flat wall Eq A.1 reduces to a fixed smoothing of the first fluid row per
layer (closed form for cosine modes on D2Q9 and D3Q19); a uniform fluid at
rest next to any solid shape, with the wall's chemical potential equal to the
fluid's, is a fixed point; halfway bounce-back leaves no normal momentum at
the first fluid row; mass is conserved; mirror symmetry is kept; and a larger
wall chemical potential wets less."""
import numpy as np
import pytest

from paper_2205_09186_amd import inputs


def _params(orc, lat, shape, scheme, solid=None, mu_wall=0.0, Tr=0.8, k=0.16, kappa=0.004, tau=1.0):
    nz, ny, nx = ((1,) + tuple(shape)) if lat == 0 else tuple(shape)
    return orc.Params(lattice=lat, nx=nx, ny=ny, nz=nz, tau=tau, Tr=Tr, k=k, kappa=kappa, scheme=scheme,
                      solid=solid, mu_wall=mu_wall)


def _mu_bulk(orc, rho, Tr, k):
    Tc, _, _ = orc.pr_critical()
    return k * k * orc.pr_mub(rho, Tr * Tc, orc.PR_A * orc.pr_alpha(Tr), orc.PR_B, orc.PR_R)


@pytest.mark.parametrize("lat,shape", [(0, (30, 26)), (1, (10, 12, 14))])
def test_all_fluid_mask_is_the_periodic_step(orc, lat, shape):
    g, l = orc.maxwell(0.8)
    rho0 = inputs.droplet(shape, min(shape) / 4, 3.0, g, l)
    a = orc.Sim(_params(orc, lat, shape, orc.CD4), rho0)
    b = orc.Sim(_params(orc, lat, shape, orc.CD4, solid=np.zeros(shape, np.uint8), mu_wall=0.3), rho0)
    a.step(20); b.step(20)
    assert np.array_equal(a.populations(), b.populations())


@pytest.mark.parametrize("scheme,r", [("CD2", 1), ("CD4", 2), ("CD6", 3)])
def test_flat_wall_layers_and_eq_a1_closed_form_d2q9(orc, scheme, r):
    """Solid rows 0..7 under fluid rows 8..: the layers are rows 7, 6, 5 from
    the fluid above and rows 0, 1, 2 from the periodic image of the top row;
    Eq A.1 with the D2Q9 weights maps a cosine mode of the neighbour row to
    the same mode times (4 + 2 cos q) / 6."""
    nx, ny, ws = 24, 30, 8
    solid = np.zeros((ny, nx), np.uint8)
    solid[:ws] = 1
    xs = np.arange(nx)
    q = 2 * np.pi * 3 / nx
    rho = np.ones((ny, nx)) * 2.0
    rho[ws] = 2.0 + 0.3 * np.cos(q * xs)          # first fluid row
    rho[ny - 1] = 1.5 - 0.2 * np.cos(2 * q * xs)  # last fluid row, next to the image wall
    p = _params(orc, 0, (ny, nx), orc.SCHEME_NAMES[scheme], solid=solid)
    out, layer = orc.wall_density(p, rho)
    for l in range(1, r + 1):
        assert np.all(layer[ws - l] == l) and np.all(layer[l - 1] == l)
        c1, c2 = ((4 + 2 * np.cos(q)) / 6) ** l, ((4 + 2 * np.cos(2 * q)) / 6) ** l
        np.testing.assert_allclose(out[ws - l], 2.0 + 0.3 * c1 * np.cos(q * xs), rtol=0, atol=1e-14)
        np.testing.assert_allclose(out[l - 1], 1.5 - 0.2 * c2 * np.cos(2 * q * xs), rtol=0, atol=1e-14)
    assert np.all(layer[r:ws - r] == -1)
    assert np.all(layer[ws:] == 0)
    np.testing.assert_array_equal(out[ws:], rho[ws:])


def test_flat_wall_eq_a1_closed_form_d3q19(orc):
    """D3Q19: the fluid neighbours of a wall node are (0,0,1) with weight 1/18
    and the four (+-1,0,1), (0,+-1,1) with 1/36, so a mode cos(q x + p y)
    is scaled by (1 + cos q + cos p) / 3 per layer."""
    nx, ny, nz, ws = 12, 10, 16, 6
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:ws] = 1
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    q, pp = 2 * np.pi * 2 / nx, 2 * np.pi / ny
    rho = np.full((nz, ny, nx), 2.0)
    rho[ws] = 2.0 + 0.25 * np.cos(q * xx + pp * yy)
    p = _params(orc, 1, (nz, ny, nx), orc.CD6, solid=solid)
    out, layer = orc.wall_density(p, rho)
    for l in (1, 2, 3):
        assert np.all(layer[ws - l] == l)
        c = ((1 + np.cos(q) + np.cos(pp)) / 3) ** l
        np.testing.assert_allclose(out[ws - l], 2.0 + 0.25 * c * np.cos(q * xx + pp * yy), rtol=0, atol=1e-14)


@pytest.mark.parametrize("lat,shape,scheme", [(0, (28, 33), "CD6"), (1, (12, 13, 14), "CD4")])
def test_uniform_rest_state_next_to_a_solid_is_a_fixed_point(orc, lat, shape, scheme):
    Tr, k, rho_u = 0.8, 0.16, 3.1
    idx = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    d2 = sum((i - s / 2 + 0.3) ** 2 for i, s in zip(idx, shape))
    solid = (d2 < (min(shape) / 4) ** 2).astype(np.uint8)      # an off-centre ball
    p = _params(orc, lat, shape, orc.SCHEME_NAMES[scheme], solid=solid, mu_wall=_mu_bulk(orc, rho_u, Tr, k),
                Tr=Tr, k=k, tau=0.8)
    s = orc.Sim(p, np.full(shape, rho_u))
    f0 = s.populations().copy()
    s.step(10)
    np.testing.assert_allclose(s.populations(), f0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("lat", [0, 1])
def test_bounce_back_leaves_no_normal_momentum(orc, lat):
    """A uniform flow towards a flat wall (tau = 1, no force since the wall's
    chemical potential equals the fluid's): after one step the first fluid
    layer on either side of the solid slab carries no momentum normal to the
    wall, and its tangential momentum is that of the populations that move
    parallel to the wall."""
    Tr, k, rho_u = 0.8, 0.16, 2.7
    shape = (20, 9) if lat == 0 else (14, 6, 7)
    solid = np.zeros(shape, np.uint8)
    solid[:4] = 1
    u = (0.03, -0.04) if lat == 0 else (0.03, 0.02, -0.04)
    p = _params(orc, lat, shape, orc.CD2, solid=solid, mu_wall=_mu_bulk(orc, rho_u, Tr, k), Tr=Tr, k=k)
    s = orc.Sim(p, np.full(shape, rho_u))
    e, w = orc.lattice(lat)
    fe = orc.feq(lat, rho_u, u)
    f = s.populations()
    fluid = solid.reshape(-1) == 0
    f[:, fluid] = fe[:, None]
    s.step(1)
    f = s.populations()
    nd = 1 if lat == 0 else 2                          # the wall-normal axis
    n = f.shape[1]
    layer_nodes = [np.arange(n).reshape(shape)[4].reshape(-1), np.arange(n).reshape(shape)[-1].reshape(-1)]
    par = e[:, nd] == 0
    for nodes in layer_nodes:
        j = e[:, :3].T.astype(float) @ f[:, nodes]
        np.testing.assert_allclose(j[nd], 0.0, atol=1e-15)
        for t in range(len(u)):
            if t != nd:
                np.testing.assert_allclose(j[t], (e[par, t] * fe[par]).sum(), rtol=1e-13)
    # away from the walls the uniform flow is untouched
    mid = np.arange(n).reshape(shape)[shape[0] // 2 + 2].reshape(-1)
    np.testing.assert_allclose(f[:, mid], np.repeat(fe[:, None], mid.size, axis=1), rtol=1e-14)


def _wall_droplet(orc, mu_wall_rel, steps, nx=96, ny=64, ws=6, scheme="CD4"):
    Tr, k = 0.8, 0.16
    g, l = orc.maxwell(Tr)
    solid = np.zeros((ny, nx), np.uint8)
    solid[:ws] = 1
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    r = np.hypot(xx - nx / 2, yy - (ws + 12))
    rho0 = (l + g) / 2 - (l - g) / 2 * np.tanh(2 * (r - 16) / 4.0)
    muM = _mu_bulk(orc, g, Tr, k)
    p = _params(orc, 0, (ny, nx), orc.SCHEME_NAMES[scheme], solid=solid,
                mu_wall=muM + mu_wall_rel * abs(muM), Tr=Tr, k=k)
    s = orc.Sim(p, rho0)
    M0 = s.observables()[1]
    s.step(steps)
    return s, M0, (l + g) / 2, ws


def test_wall_conserves_mass_and_keeps_mirror_symmetry(orc):
    s, M0, mid, ws = _wall_droplet(orc, 1.0, 600)
    U, M = s.observables()
    assert abs(M - M0) < 1e-13 * M0
    rho = s.macros()[0]
    # droplet centred at x = nx/2 on the node grid: x -> nx - x is a symmetry
    np.testing.assert_allclose(rho[:, 1:], rho[:, 1:][:, ::-1], rtol=0, atol=1e-12)
    assert np.all(rho[:ws] == 0.0)


def test_larger_wall_chemical_potential_wets_less(orc):
    """The wall chemical potential sets the wettability (Appendix): with
    mu_wall above the coexistence value the force near the wall points away
    from it, so the droplet's footprint on the wall shrinks and it stands
    taller; below, it spreads."""
    foot, height = [], []
    for rel in (-3.0, 0.0, 6.0):
        s, _, mid, ws = _wall_droplet(orc, rel, 1500)
        rho = s.macros()[0]
        foot.append(int((rho[ws] > mid).sum()))
        height.append(int((rho[:, rho.shape[1] // 2] > mid).sum()))
    assert foot[0] > foot[1] > foot[2], foot
    assert height[0] < height[2], height


def test_walls_need_a_central_scheme(orc):
    solid = np.zeros((10, 12), np.uint8)
    solid[:3] = 1
    for sch in (orc.E4, orc.OCFDS4, orc.CFDS6):
        p = _params(orc, 0, (10, 12), sch, solid=solid)
        with pytest.raises(ValueError):
            orc.Sim(p, np.full((10, 12), 2.0))
