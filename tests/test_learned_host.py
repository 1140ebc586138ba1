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
