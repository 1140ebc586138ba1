"""Pins of the oracle's D2Q9 MRT collision (Eq 1, 3, 4, 5 with EDM forcing,
Eq 8), each against something other than the oracle's own arithmetic."""
import numpy as np
import pytest

from paper_2205_09186_amd import inputs


def test_matrix_rows_orthogonal_and_inverse(orc):
    """Eq 3 calls M orthogonal: M M^T is diagonal with the squared row norms
    of the moment basis (9, 36, 36, 6, 12, 6, 12, 4, 4); the oracle's inverse
    is a true inverse."""
    M, Mi = orc.mrt_matrix()
    G = M @ M.T
    np.testing.assert_array_equal(G, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]).astype(float))
    np.testing.assert_allclose(M @ Mi, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(Mi, M.T / np.diag(G)[None, :], atol=1e-16)


def test_matrix_rows_are_the_named_moments(orc):
    """Rows 1, 4, 6 are density and momentum over the directions of Eq 2; the
    equilibrium moments of Eq 6 take the closed forms of the D2Q9 moment
    basis: e = -2 rho + 3 rho u^2, eps = rho - 3 rho u^2, q = -rho u,
    p_xx = rho (ux^2 - uy^2), p_xy = rho ux uy."""
    M, _ = orc.mrt_matrix()
    e, _ = orc.lattice(orc.D2Q9)
    np.testing.assert_array_equal(M[0], np.ones(9))
    np.testing.assert_array_equal(M[3], e[:, 0])
    np.testing.assert_array_equal(M[5], e[:, 1])
    rng = np.random.default_rng(7)
    for _ in range(20):
        rho = rng.uniform(0.01, 8.0)
        ux, uy = rng.uniform(-0.1, 0.1, 2)
        m = M @ orc.feq(orc.D2Q9, rho, (ux, uy))
        u2 = ux * ux + uy * uy
        want = [rho, -2 * rho + 3 * rho * u2, rho - 3 * rho * u2, rho * ux, -rho * ux, rho * uy, -rho * uy,
                rho * (ux * ux - uy * uy), rho * ux * uy]
        np.testing.assert_allclose(m, want, rtol=1e-13, atol=1e-14 * rho)


def test_reduces_to_srt(orc):
    """Sec 2.1: with every rate 1/tau the MRT model is the SRT model."""
    rng = np.random.default_rng(3)
    for tau in (0.6, 1.0, 1.7):
        for _ in range(10):
            f = orc.feq(orc.D2Q9, rng.uniform(0.5, 5), rng.uniform(-0.05, 0.05, 2)) * (1 + 0.01 * rng.standard_normal(9))
            F = rng.uniform(-1e-3, 1e-3, 2)
            a = orc.collide_node_mrt(tau, f, F, s_e=1 / tau, s_eps=1 / tau, s_q=1 / tau)
            b = orc.collide_node(orc.D2Q9, tau, f, list(F) + [0.0])
            np.testing.assert_allclose(a, b, rtol=0, atol=4e-15 * f.sum())


def test_each_moment_relaxes_with_its_rate(orc):
    """Without force, (m* - m_eq) = (1 - s_k)(m - m_eq) row by row, with the
    rates of Sec 2.1 in the row order of Eq 3 and Eq 5; conserved moments keep
    their values."""
    M, _ = orc.mrt_matrix()
    rng = np.random.default_rng(11)
    tau = 0.8
    s = np.array([1.0, 1.64, 1.54, 1.0, 1.7, 1.0, 1.7, 1 / tau, 1 / tau])
    for _ in range(10):
        rho = rng.uniform(0.5, 5)
        u = rng.uniform(-0.05, 0.05, 2)
        f = orc.feq(orc.D2Q9, rho, u) + 0.01 * rho * rng.standard_normal(9) * np.array([0, 1, 1, 1, 1, 1, 1, 1, 1])
        # put the perturbation outside the conserved moments
        Mi = np.linalg.inv(M)
        m = M @ f
        m[[0, 3, 5]] = (M @ orc.feq(orc.D2Q9, rho, u))[[0, 3, 5]]
        f = Mi @ m
        out = orc.collide_node_mrt(tau, f, (0.0, 0.0))
        r = f.sum()
        ueq = np.array([(M[3] @ f) / r, (M[5] @ f) / r])
        meq = M @ orc.feq(orc.D2Q9, r, ueq)
        np.testing.assert_allclose(M @ out - meq, (1 - s) * (M @ f - meq), atol=2e-15 * r)


def test_edm_momentum_and_mass(orc):
    """Sum f* = sum f and sum e f* = sum e f + F (Eq 7, 8) under MRT."""
    e, _ = orc.lattice(orc.D2Q9)
    rng = np.random.default_rng(5)
    for _ in range(20):
        f = orc.feq(orc.D2Q9, rng.uniform(0.5, 5), rng.uniform(-0.05, 0.05, 2)) * (1 + 0.02 * rng.standard_normal(9))
        F = rng.uniform(-1e-2, 1e-2, 2)
        out = orc.collide_node_mrt(0.9, f, F)
        assert out.sum() == pytest.approx(f.sum(), rel=1e-15)
        np.testing.assert_allclose(e[:, :2].T @ out, e[:, :2].T @ f + F, atol=2e-15 * f.sum())


def test_step_mrt_with_srt_rates_equals_srt(orc):
    """Whole steps: MRT with every rate 1/tau follows the SRT oracle."""
    g, l = orc.maxwell(0.9)
    rho0 = inputs.droplet((40, 36), 9, 4.0, g, l)
    kw = dict(lattice=orc.D2Q9, nx=36, ny=40, tau=0.8, Tr=0.9, k=0.16, kappa=0.004, scheme=orc.CD4)
    a = orc.Sim(orc.Params(**kw, collision=1, s_e=1.25, s_eps=1.25, s_q=1.25), rho0)
    b = orc.Sim(orc.Params(**kw), rho0)
    a.step(50); b.step(50)
    assert np.abs(a.macros()[0] - b.macros()[0]).max() < 1e-13


def test_step_mrt_conserves_mass(orc):
    g, l = orc.maxwell(0.8)
    rho0 = inputs.droplet((60, 60), 15, 4.0, g, l)
    p = orc.Params(lattice=orc.D2Q9, nx=60, ny=60, tau=1.0, Tr=0.8, k=0.16, kappa=0.004, scheme=orc.CD4, collision=1)
    s = orc.Sim(p, rho0)
    m0 = s.observables()[1]
    s.step(2000)
    U, m = s.observables()
    assert np.isfinite(U)
    assert abs(m - m0) / m0 < 1e-13
