"""Host logic of the learned initialiser (no GPU)."""


def test_learned_3d_droplet_set_is_seeded_and_box_relative():
    """The 3D droplets of the learned-start comparison: reproducible from the
    seed, radius a fixed fraction of the box, temperatures in each scheme's
    range."""
    from paper_2205_09186_amd import learned, lbm
    a = learned.droplet_set_3d(12, 7)
    b = learned.droplet_set_3d(12, 7)
    assert a == b
    assert a != learned.droplet_set_3d(12, 8)
    for d in a:
        assert d["L"] in (96, 128)
        assert 0.22 * d["L"] <= d["R"] <= 0.32 * d["L"]
        lo, hi = learned.STABLE_TR.get(d["scheme"], (0.65, 0.85))
        assert lo <= d["Tr"] <= hi
        assert 0.1 <= d["k"] <= 0.25


def test_gain_summary_accounting():
    """The learned-vs-tanh summary compares only droplets whose two runs met the
    criterion and still hold a droplet, and counts the steps saved over every
    droplet whose two runs met it (a run stopped at the cap, or one that
    diverged, counts in neither)."""
    import pytest
    from paper_2205_09186_amd import learned, lbm
    C, RUN, DIV = lbm.CONVERGED, lbm.RUNNING, lbm.DIVERGED
    specs = [dict(L=64, R=16.0, scheme=2, Tr=0.7, k=0.1)] * 5
    drop, gas = (8.0, 0.2), (0.3, 0.25)
    t = ([C, C, RUN, C, C], [1000, 500, 400000, 900, 2000], [1e-5, 3e-6, 4e-6, 5e-6, 2e-5],
         [drop, gas, drop, drop, drop], 1.0, "tanh mode")
    lrn = ([C, C, C, DIV, C], [800, 400, 40000, 10, 2100], [1e-5 * (1 + 1e-7), 3e-6, 4e-6, 0.0, 2e-5 * (1 + 3e-7)],
           [drop, gas, drop, drop, (8.0 * (1 + 2e-9), 0.2 * (1 + 5e-9))], 2.0, "learned mode")
    sm, rows = learned.gain_summary(specs, 1, t, lrn)
    assert sm["droplets"] == 5 and sm["fallback"] == 1
    assert sm["compared"] == 2 and [("ratio" in r) for r in rows] == [True, False, False, False, True]
    assert sm["steps_ratio_median"] == pytest.approx((0.8 + 1.05) / 2)
    assert sm["learned_fewer_steps"] == 1
    assert sm["both_converged"] == 3
    assert sm["steps_saved_total"] == pytest.approx(1 - (800 + 400 + 2100) / (1000 + 500 + 2000))
    assert sm["not_converged"] == {"tanh": 1, "learned": 1}
    assert sm["U_reldiff_max"] == pytest.approx(3e-7, rel=1e-6)
    assert sm["U_within_1e6"] == 2
    assert sm["rho_l_reldiff_max"] == pytest.approx(2e-9, rel=1e-6)
    assert sm["rho_g_reldiff_max"] == pytest.approx(5e-9, rel=1e-6)
    assert rows[2]["status"] == (RUN, C) and rows[3]["steps"] == (900, 10)
