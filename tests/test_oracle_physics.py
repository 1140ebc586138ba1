"""Pins of the oracle's lattice kinetics (Sec 2.1), thermodynamics (Sec 2.2) and
full step against identities and closed forms the paper and mathematics fix."""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
from scipy import integrate

from paper_2205_09186_amd import inputs


# --------------------------------------------------------------------------- #
# Lattices and equilibrium (Eq 2, Eq 6, Eq 7)                                   #
# --------------------------------------------------------------------------- #
def test_d2q9_directions_follow_eq2(orc):
    e, w = orc.lattice(orc.D2Q9)
    expect = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    assert [tuple(v[:2]) for v in e] == expect
    np.testing.assert_allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=2.5e-16, atol=0)
    # the rounded weights sum to one exactly (no systematic mass change)
    from fractions import Fraction
    assert sum(Fraction(x) for x in w) == 1


@pytest.mark.parametrize("lat", [0, 1])
def test_lattice_isotropy(orc, lat):
    e, w = orc.lattice(lat)
    dim = 2 if lat == 0 else 3
    e = e[:, :dim].astype(float)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, e, e), np.eye(dim) / 3, atol=1e-15)
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    d = np.eye(dim)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    np.testing.assert_allclose(M4, iso, atol=1e-15)


@pytest.mark.parametrize("lat", [0, 1])
def test_feq_moments(orc, lat):
    e, _ = orc.lattice(lat)
    dim = 2 if lat == 0 else 3
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho = rng.uniform(0.01, 9.0)
        u = rng.uniform(-0.1, 0.1, 3)
        u[dim:] = 0.0
        fe = orc.feq(lat, rho, u)
        assert fe.sum() == pytest.approx(rho, rel=1e-14)
        np.testing.assert_allclose(e.T @ fe, rho * u, atol=1e-14 * rho)
        P = np.einsum("i,ia,ib->ab", fe, e[:, :dim], e[:, :dim])
        np.testing.assert_allclose(P, rho / 3 * np.eye(dim) + rho * np.outer(u[:dim], u[:dim]), atol=1e-13 * rho)


@pytest.mark.parametrize("lat", [0, 1])
def test_edm_collision_identities(orc, lat):
    """Eq 8: sum_i F_i = 0 and sum_i e_i F_i = rho du = F; tau = 1 gives
    f* = feq(rho, u + du) exactly (SRT reduction of Eq 1)."""
    e, _ = orc.lattice(lat)
    dim = 2 if lat == 0 else 3
    q = len(e)
    rng = np.random.default_rng(11)
    for tau in (0.8, 1.0, 1.7):
        f = orc.feq(lat, 3.0, [0.02, -0.01, 0.015][:dim]) * (1 + 0.05 * rng.standard_normal(q))
        F = np.array([0.003, -0.002, 0.001])
        F[dim:] = 0.0
        fs = orc.collide_node(lat, tau, f, F)
        rho = f.sum()
        assert fs.sum() == pytest.approx(rho, rel=1e-14)
        np.testing.assert_allclose(e.T @ fs, e.T @ f + F, atol=1e-15)
        if tau == 1.0:
            u = (e.T @ f) / rho
            np.testing.assert_allclose(fs, orc.feq(lat, rho, u + F / rho), atol=1e-15)
        # a relaxed (equilibrium) state without force is a fixed point
        fe = orc.feq(lat, rho, (e.T @ f) / rho)
        np.testing.assert_allclose(orc.collide_node(lat, tau, fe, [0, 0, 0]), fe, atol=1e-15)


# --------------------------------------------------------------------------- #
# Peng-Robinson EOS (Eq 13-15)                                                  #
# --------------------------------------------------------------------------- #
def test_pr_critical_point(orc):
    Tc, rc, pc = orc.pr_critical()
    a, b, R = orc.PR_A, orc.PR_B, orc.PR_R
    h = 1e-4 * rc
    p = lambda r: orc.pr_p0(r, Tc, a, b, R)
    d1 = (p(rc + h) - p(rc - h)) / (2 * h)
    d2 = (p(rc + h) - 2 * p(rc) + p(rc - h)) / h ** 2
    assert abs(d1) < 1e-9 and abs(d2) < 1e-7
    # textbook Peng-Robinson constants: a = 0.45724 R^2 Tc^2/pc, b = 0.07780 R Tc/pc, Zc = 0.3074
    assert a * pc / (R * Tc) ** 2 == pytest.approx(0.45724, rel=2e-5)
    assert b * pc / (R * Tc) == pytest.approx(0.07780, rel=2e-4)
    assert pc / (rc * R * Tc) == pytest.approx(0.3074, rel=2e-4)
    # above Tc the isotherm is monotone: no coexistence
    with pytest.raises(ValueError):
        orc.maxwell(1.0)


def test_pr_alpha_and_gibbs_duhem(orc):
    Tc, rc, pc = orc.pr_critical()
    assert orc.pr_alpha(1.0) == 1.0
    b, R = orc.PR_B, orc.PR_R
    for Tr in (0.3, 0.6, 0.9):
        T = Tr * Tc
        aa = orc.PR_A * orc.pr_alpha(Tr)
        for rho in (1e-6, 0.05, 1.3, 4.0, 9.5):
            h = 1e-6 * rho
            dmu = (orc.pr_mub(rho + h, T, aa) - orc.pr_mub(rho - h, T, aa)) / (2 * h)
            dp = (orc.pr_p0(rho + h, T, aa) - orc.pr_p0(rho - h, T, aa)) / (2 * h)
            assert dmu == pytest.approx(dp / rho, rel=1e-7, abs=1e-9)


def test_pr_free_energy_eq10_eq13(orc):
    """psi = rho (int p0/rho^2 drho + C) (Eq 13) by quadrature; then
    p0 = rho psi' - psi (Eq 10) with psi' the oracle's mu_b, C chosen so the two
    agree at one density."""
    Tc, _, _ = orc.pr_critical()
    Tr = 0.7
    T, aa = Tr * Tc, orc.PR_A * orc.pr_alpha(Tr)
    r0 = 1.0
    # fix C from Eq 10 at r0
    C0 = (r0 * orc.pr_mub(r0, T, aa) - orc.pr_p0(r0, T, aa)) / r0
    for rho in (0.2, 2.5, 7.0):
        I, _ = integrate.quad(lambda r: orc.pr_p0(r, T, aa) / r ** 2, r0, rho, epsabs=1e-14, epsrel=1e-13)
        psi = rho * (I + C0)
        assert rho * orc.pr_mub(rho, T, aa) - psi == pytest.approx(orc.pr_p0(rho, T, aa), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("Tr", [0.95, 0.9, 0.8, 0.7, 0.6, 0.5, 0.4, 0.3, 0.25, 0.2])
def test_maxwell_two_formulations(orc, Tr):
    g1, l1 = orc.maxwell(Tr, "mu")
    g2, l2 = orc.maxwell(Tr, "area")
    assert g1 == pytest.approx(g2, rel=2e-12)
    assert l1 == pytest.approx(l2, rel=1e-13)
    Tc, rc, _ = orc.pr_critical()
    assert g1 < rc < l1
    T, aa = Tr * Tc, orc.PR_A * orc.pr_alpha(Tr)
    # the liquid pressure is a difference of O(1) terms: compare on their scale
    scale = l1 * orc.PR_R * T / (1 - orc.PR_B * l1)
    assert abs(orc.pr_p0(g1, T, aa) - orc.pr_p0(l1, T, aa)) < 1e-13 * scale
    assert orc.pr_mub(g1, T, aa) == pytest.approx(orc.pr_mub(l1, T, aa), rel=1e-12)


def _golden_maxwell():
    """(critical point dict, rows (Tr, rho_g, rho_l) as strings) of tests/golden/maxwell_pr.txt."""
    import os
    crit, rows = {}, []
    with open(os.path.join(os.path.dirname(__file__), "golden", "maxwell_pr.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].split()
            if len(line) == 2:
                crit[line[0]] = line[1]
            elif len(line) == 3:
                rows.append(tuple(line))
    return crit, rows


def _digits_tol(s: str) -> float:
    """Half a unit in the last significant digit of a printed number, or 1e-9
    relative when more than nine significant digits are printed."""
    mant = s.lower().split("e")[0].replace("-", "").replace(".", "").lstrip("0")
    v = abs(float(s))
    sig = len(mant)
    if sig > 9:
        return 1e-9 * v
    return 0.51 * 10.0 ** (math.floor(math.log10(v)) - sig + 1)


def test_critical_point_against_independent_values(orc):
    crit, _ = _golden_maxwell()
    Tc, rc, pc = orc.pr_critical()
    for name, val in (("Tc", Tc), ("rho_c", rc), ("p_c", pc)):
        assert abs(val - float(crit[name])) <= _digits_tol(crit[name]), (name, val, crit[name])


def test_maxwell_against_independent_table(orc):
    """Coexistence densities from T_r = 0.95 down to 0.2 against an independent
    computation from the paper's formulas.  Both of the oracle's Maxwell
    formulations share p0 and alpha(T), so this is what pins alpha(T)'s
    acentric polynomial (a slip in it shifts every row by far more than the
    tolerance)."""
    _, rows = _golden_maxwell()
    assert len(rows) == 10
    for Tr, g_s, l_s in rows:
        for method in ("mu", "area"):
            g, l = orc.maxwell(float(Tr), method)
            assert abs(g - float(g_s)) <= _digits_tol(g_s), (Tr, method, g, g_s)
            assert abs(l - float(l_s)) <= _digits_tol(l_s), (Tr, method, l, l_s)


@pytest.mark.parametrize("omega", [0.0, 0.2, 0.344, 0.5])
def test_acentric_factor_definition(orc, omega):
    """Pitzer's definition of the acentric factor, omega = -1 - log10(p_sat/p_c)
    at T_r = 0.7, is what the temperature function alpha(T) of the
    Peng-Robinson EOS (Sec 2.2) is fitted to reproduce: with the oracle's alpha
    the EOS's own saturation pressure gives back the omega it was given, to the
    few thousandths the correlation achieves."""
    Tc, _, pc = orc.pr_critical()
    g, _ = orc.maxwell(0.7, omega=omega)
    aa = orc.PR_A * orc.pr_alpha(0.7, omega)
    psat = orc.pr_p0(g, 0.7 * Tc, aa)
    assert -1.0 - math.log10(psat / pc) == pytest.approx(omega, abs=5e-3)
    # alpha(Tc) = 1 for any omega, and alpha falls with temperature
    assert orc.pr_alpha(1.0, omega) == 1.0
    if omega > 0:
        assert orc.pr_alpha(0.5, omega) > orc.pr_alpha(0.7, omega) > 1.0


def test_maxwell_density_ratio_trend(orc):
    """Sec 3.3: the density ratio grows as the temperature falls; Sec 4 quotes
    ratios up to ~1000 for the droplet runs (T_r = 0.6 is near 850)."""
    ratios = [orc.maxwell(t)[1] / orc.maxwell(t)[0] for t in (0.9, 0.8, 0.7, 0.6)]
    assert all(b > a for a, b in zip(ratios, ratios[1:]))
    assert 500 < ratios[-1] < 1500


# --------------------------------------------------------------------------- #
# Full step: invariants                                                         #
# --------------------------------------------------------------------------- #
def _droplet_sim(orc, lat, n, scheme, Tr=0.8, k=0.16, kappa=0.004, W=2.0, R=None, amp=1e-6):
    g, l = orc.maxwell(Tr)
    if lat == orc.D2Q9:
        p = orc.Params(lattice=lat, nx=n, ny=n, nz=1, Tr=Tr, k=k, kappa=kappa, scheme=scheme)
        rho0 = inputs.droplet((n, n), R or n / 4, W, g, l, amplitude=amp)
    else:
        p = orc.Params(lattice=lat, nx=n, ny=n, nz=n, Tr=Tr, k=k, kappa=kappa, scheme=scheme)
        rho0 = inputs.droplet((n, n, n), R or n / 4, W, g, l, amplitude=amp)
    return orc.Sim(p, rho0), rho0


def test_mass_conservation_2000_steps(orc):
    s, rho0 = _droplet_sim(orc, orc.D2Q9, 100, orc.CD4)
    _, m0 = s.observables()
    s.step(2000)
    u, m = s.observables()
    assert np.isfinite(u)
    assert abs(m - m0) / m0 < 1e-13


@pytest.mark.parametrize("scheme", ["CD6", "E8", "OCFDS4"])
def test_mass_conservation_3d(orc, scheme):
    s, _ = _droplet_sim(orc, orc.D3Q19, 16, orc.SCHEME_NAMES[scheme], Tr=0.9, W=4.0)
    _, m0 = s.observables()
    s.step(20)
    _, m = s.observables()
    assert abs(m - m0) / m0 < 1e-14


@pytest.mark.parametrize("lat", [0, 1])
@pytest.mark.parametrize("scheme", ["CD2", "CD6", "E8", "OCFDS4"])
def test_uniform_state_is_fixed_point(orc, lat, scheme):
    n = 12
    p = orc.Params(lattice=lat, nx=n, ny=n - 2, nz=(1 if lat == 0 else n + 1), Tr=0.7, k=0.2, kappa=0.004,
                   scheme=orc.SCHEME_NAMES[scheme])
    rho0 = np.full(p.n, 3.3)
    s = orc.Sim(p, rho0)
    f0 = s.f.copy()
    s.step(3)
    np.testing.assert_allclose(s.f, f0, rtol=0, atol=4e-15)
    r, vx, vy, vz = s.macros()
    assert np.abs(vx).max() < 1e-16 and np.abs(vy).max() < 1e-16


@pytest.mark.parametrize("lat,scheme", [(0, "CD4"), (0, "OCFDS4"), (1, "CD6")])
def test_restart_is_bitwise(orc, lat, scheme):
    """The step is a function of the post-streaming populations alone: a
    simulation given another's populations after 30 steps continues exactly
    as that one does (no state outside f carries over between steps)."""
    n = 24 if lat == 0 else 12
    a, rho0 = _droplet_sim(orc, lat, n, orc.SCHEME_NAMES[scheme], Tr=0.9, W=4.0)
    a.step(30)
    saved = a.f.copy()
    b, _ = _droplet_sim(orc, lat, n, orc.SCHEME_NAMES[scheme], Tr=0.9, W=6.0)   # same parameters, other start
    b.step(7)
    b.f[:] = saved
    a.step(20)
    b.step(20)
    assert np.array_equal(a.f, b.f)
    assert not np.array_equal(a.f, saved)


def test_droplet_symmetry_2d(orc):
    """A centred, noise-free droplet on an even grid keeps the square's symmetry."""
    s, _ = _droplet_sim(orc, orc.D2Q9, 40, orc.CD4, amp=0.0, W=4.0)
    s.step(100)
    r, vx, vy, _ = s.macros()
    # centre at node 20: reflect x -> 40 - x about node 20
    rr = np.roll(r[:, ::-1], 1, axis=1)
    np.testing.assert_allclose(r, rr, atol=1e-12)
    np.testing.assert_allclose(r, r.T, atol=1e-12)
    np.testing.assert_allclose(vx, -np.roll(vx[:, ::-1], 1, axis=1), atol=1e-12)
    np.testing.assert_allclose(vx, vy.T, atol=1e-12)


def test_droplet_symmetry_3d(orc):
    s, _ = _droplet_sim(orc, orc.D3Q19, 16, orc.CD4, Tr=0.9, amp=0.0, W=4.0)
    s.step(10)
    r, vx, vy, vz = s.macros()
    np.testing.assert_allclose(r, r.transpose(0, 2, 1), atol=1e-12)
    np.testing.assert_allclose(r, r.transpose(2, 1, 0), atol=1e-12)
    np.testing.assert_allclose(vx, vy.transpose(0, 2, 1), atol=1e-12)
    np.testing.assert_allclose(vx, vz.transpose(2, 1, 0), atol=1e-12)


def test_spurious_currents_stay_below_sound_speed(orc):
    s, _ = _droplet_sim(orc, orc.D2Q9, 64, orc.CD6, Tr=0.8)
    s.step(500)
    u, _ = s.observables()
    assert 0 < u < 0.05


# --------------------------------------------------------------------------- #
# The force that the step applies (Eq 12, Eq 16), read back from one step      #
# --------------------------------------------------------------------------- #
# Fourier symbols of the schemes on exp(i q x): the gradient multiplies by
# i*lam1(q) (Eq 28), the Laplacian by -lam2(q): the matched-order central
# second difference for the explicit schemes, lam1^2 for the compact ones,
# whose Laplacian is D(D).
_CD1 = {"CD2": (1.0, 0.0, 0.0), "CD6": (1.5, -0.6, 0.1)}
_CD2ND = {"CD2": (-2.0, 1.0), "CD6": (-490 / 180, 270 / 180, -27 / 180, 2 / 180)}


def _symbols(orc, name, q):
    if name in _CD1:
        a, b, c = _CD1[name]
        lam1 = a * np.sin(q) + b / 2 * np.sin(2 * q) + c / 3 * np.sin(3 * q)
        cs = _CD2ND[name]
        lam2 = -(cs[0] + sum(2 * cs[k] * np.cos(k * q) for k in range(1, len(cs))))
        return lam1, lam2
    al, a, b, c = orc.compact_coeffs(orc.SCHEME_NAMES[name])
    lam1 = (a * np.sin(q) + b / 2 * np.sin(2 * q) + c / 3 * np.sin(3 * q)) / (1 + 2 * al * np.cos(q))
    return lam1, lam1 ** 2


def _step_force(orc, lat, shape, scheme, rho0, k, kappa, tau):
    """Force applied by one oracle step from rest, read from the populations:
    the post-collision values at x are the post-streaming values at x + e_i,
    and their momentum is rho u + F = F (Eq 1, 6, 8: the EDM adds
    feq(rho, u + F/rho) - feq(rho, u), whose momentum is F)."""
    nz, ny, nx = shape
    p = orc.Params(lattice=lat, nx=nx, ny=ny, nz=nz, tau=tau, Tr=0.7, k=k, kappa=kappa,
                   scheme=orc.SCHEME_NAMES[scheme])
    s = orc.Sim(p, rho0)
    s.step(1)
    e, _ = orc.lattice(lat)
    f = s.populations().reshape((len(e),) + shape)
    mom = np.zeros((3,) + shape)
    rho = np.zeros(shape)
    for i, (ex, ey, ez) in enumerate(e):
        fs = np.roll(f[i], (-ez, -ey, -ex), axis=(0, 1, 2))
        rho += fs
        mom += np.array([ex, ey, ez])[:, None, None, None] * fs
    return rho, mom


@pytest.mark.parametrize("lat,scheme,axis,m", [(0, "CD2", 1, 1), (0, "CD6", 1, 3), (0, "OCFDS4", 1, 2),
                                               (1, "CD6", 0, 1), (1, "OCFDS4", 2, 3)])
def test_step_force_follows_eq12_and_eq16(orc, lat, scheme, axis, m):
    """On rho = A + B cos(q s) along one axis s, the force of one step is
    F_s = k^2 P(s) + kappa_hat K(s) + C(s) with
      K = rho B lam1 lam2 sin(q s)      (from -rho grad(-kappa_hat lap rho)),
      C = -cs^2 B lam1 sin(q s)         (from cs^2 grad rho),
    and P = -rho grad(psi'(rho)) independent of k and kappa_hat (Eq 12, 16).
    Three values of k and two of kappa_hat separate the parts: the k^2
    dependence (a k in place of k^2 fails the third k), the size and sign of
    the kappa_hat and cs^2 parts against the closed forms, and the density is
    unchanged by the collision."""
    shape = (1, 16, 4) if lat == 0 else (12, 6, 6)
    if lat == 0:
        axis_len, ax = shape[1], 1          # y of a (1, ny, nx) array
    else:
        axis_len, ax = shape[2 - axis], 2 - axis
    q = 2 * np.pi * m / axis_len
    s = np.arange(axis_len)
    A, B = 3.0, 1.0
    prof = A + B * np.cos(q * s)
    bshape = [1, 1, 1]
    bshape[ax] = axis_len
    rho0 = np.broadcast_to(prof.reshape(bshape), shape).copy()
    comp = 1 if lat == 0 else axis           # force component along s
    ks, kap = (0.1, 0.2, 0.35), (0.004, 0.02)
    F = {}
    for k, kp in [(ks[0], kap[0]), (ks[1], kap[0]), (ks[2], kap[0]), (ks[0], kap[1])]:
        rho, mom = _step_force(orc, lat, shape, scheme, rho0, k, kp, tau=0.8)
        np.testing.assert_allclose(rho, rho0, rtol=0, atol=1e-14)
        # no force across the wave
        for d in range(3):
            if d != comp:
                assert np.abs(mom[d]).max() < 1e-15
        F[(k, kp)] = mom[comp]
    P = (F[(ks[1], kap[0])] - F[(ks[0], kap[0])]) / (ks[1] ** 2 - ks[0] ** 2)
    scale = np.abs(F[(ks[2], kap[0])]).max()
    np.testing.assert_allclose(F[(ks[2], kap[0])], F[(ks[0], kap[0])] + (ks[2] ** 2 - ks[0] ** 2) * P,
                               rtol=0, atol=1e-12 * scale)
    lam1, lam2 = _symbols(orc, scheme, q)
    sin = np.broadcast_to(np.sin(q * s).reshape(bshape), shape)
    K = (F[(ks[0], kap[1])] - F[(ks[0], kap[0])]) / (kap[1] - kap[0])
    K_exact = rho0 * B * lam1 * lam2 * sin
    np.testing.assert_allclose(K, K_exact, rtol=0, atol=1e-9 * np.abs(K_exact).max())
    C = F[(ks[0], kap[0])] - ks[0] ** 2 * P - kap[0] * K
    C_exact = -B * lam1 * sin / 3.0
    np.testing.assert_allclose(C, C_exact, rtol=0, atol=1e-11 * np.abs(C_exact).max())
    # the EOS part pulls towards the dense phase: P has the sign of -rho' psi''
    assert np.abs(P).max() > 0


# --------------------------------------------------------------------------- #
# Flat interface against the Maxwell construction (Sec 3.4, Fig 13)             #
# --------------------------------------------------------------------------- #
# The paper's flat-interface run: a layer of liquid across the middle of a
# periodic column of height 400, tau = 0.8, k = 0.1, 150,000 steps.  kappa_hat
# is not printed; 0.004 is the reading used throughout.  The column is one node
# wide: the state depends on the height only.
_SLAB_H, _SLAB_STEPS = 400, 150000
_SLAB_CASES = [(s, t) for s in ("CD6", "OCFDS4") for t in (0.9, 0.8, 0.7, 0.6)]


def _slab_run(args):
    import oracle as orc
    scheme, Tr, H, steps, tau = args
    orc.set_threads(1)          # this worker thread's own OpenMP setting
    g, l = orc.maxwell(Tr)
    p = orc.Params(nx=1, ny=H, tau=tau, Tr=Tr, k=0.1, kappa=0.004, scheme=orc.SCHEME_NAMES[scheme])
    s = orc.Sim(p, inputs.slab((H, 1), 0, 10.0, g, l, amplitude=0.0))
    s.step(steps)
    r, vx, vy, _ = s.macros()
    return (r[H // 2, 0] - l) / l, (r[0, 0] - g) / g, np.abs(vy).max()


@pytest.fixture(scope="module")
def paper_slabs(orc):
    """The eight flat-interface runs, each on one thread, run side by side."""
    with ThreadPoolExecutor(max_workers=len(_SLAB_CASES)) as ex:
        res = list(ex.map(_slab_run, [(s, t, _SLAB_H, _SLAB_STEPS, 0.8) for s, t in _SLAB_CASES]))
    return dict(zip(_SLAB_CASES, res))


@pytest.mark.slow
@pytest.mark.parametrize("scheme", ["CD6", "OCFDS4"])
@pytest.mark.parametrize("Tr", [0.9, 0.8, 0.7])
def test_flat_interface_coexistence_vs_maxwell(paper_slabs, scheme, Tr):
    """Sec 3.4 / Fig 13: at the paper's flat-interface geometry both coexistence
    densities agree with the Maxwell construction: the liquid to 1e-3, the gas
    to 1e-2 (measured: liquid within 5e-4, gas within 0.06-0.5 %)."""
    el, eg, U = paper_slabs[(scheme, Tr)]
    assert U < 1e-4
    assert abs(el) < 1e-3
    assert abs(eg) < 1e-2


@pytest.mark.slow
@pytest.mark.parametrize("scheme,bound", [("CD6", 0.03), ("OCFDS4", 0.06)])
def test_flat_interface_gas_offset_at_tr06(paper_slabs, scheme, bound):
    """At T_r = 0.6 (density ratio ~850) the liquid still agrees to 1e-3 and
    the gas density lies a few per cent above Maxwell, further for OCFDS4 than
    for CD6 (measured +1.6 % and +4.1 %): recorded, not claimed as agreement."""
    el, eg, U = paper_slabs[(scheme, 0.6)]
    assert abs(el) < 1e-3
    assert 0.0 < eg < bound


def _slab_short(orc, scheme, Tr, steps=24000, H=160):
    g, l = orc.maxwell(Tr)
    p = orc.Params(nx=1, ny=H, Tr=Tr, k=0.1, kappa=0.004, scheme=orc.SCHEME_NAMES[scheme])
    s = orc.Sim(p, inputs.slab((H, 1), 0, 10.0, g, l, amplitude=0.0))
    s.step(steps)
    r, vx, vy, _ = s.macros()
    return (r[H // 2, 0] - l) / l, (r[0, 0] - g) / g, np.abs(vy).max()


def test_flat_interface_isotropic_deviates_more(orc):
    """Sec 3.4: the coexistence densities of E4 deviate from the Maxwell curve
    more than those of the fourth-order schemes (a trend; a shorter column)."""
    el4, eg4, _ = _slab_short(orc, "E4", 0.9)
    elc, egc, _ = _slab_short(orc, "CD4", 0.9)
    assert abs(el4) > 5 * abs(elc)
