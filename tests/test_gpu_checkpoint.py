"""Checkpoint and restart through the C-ABI (lbm_save_state / lbm_load_state):
a context loaded from an image continues bitwise as the saved run, for the
launch designs (2D fused collide, 3D ring and tile collides with both
marches, compact schemes, the node-parallel path, MRT, the wetting boundary),
with the image in host or device memory; images of another grid, images that
are not images, and batch instances are refused."""
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


def _case(L, orc, lat, shape, scheme, coll=0, wall=False):
    Tr = 0.9 if scheme in ("CD2", "E8") else 0.8
    g, l = orc.maxwell(Tr)
    rho0 = inputs.droplet(shape, min(shape[-2:]) / 4, 4.0, g, l)
    nz, ny, nx = ((1,) + shape) if lat == 0 else shape
    kw = dict(lattice=lat, nx=nx, ny=ny, nz=nz, Tr=Tr, k=0.16, kappa=0.004, scheme=L.SCHEMES[scheme],
              collision=coll)
    solid = None
    if wall:
        solid = np.zeros(shape, np.uint8)
        solid[:4] = 1
        Tc, _, _ = orc.pr_critical()
        kw.update(wall=1, mu_wall=0.16 ** 2 * orc.pr_mub(g, Tr * Tc, orc.PR_A * orc.pr_alpha(Tr), orc.PR_B, orc.PR_R))
    return L.Params(**kw), rho0, solid


@pytest.mark.parametrize("lat,shape,scheme,coll,wall,nofused", [
    (0, (100, 100), "CD4", 0, False, False), (0, (40, 44), "OCFDS4", 0, False, False),
    (0, (48, 50), "CD6", 1, False, False), (0, (64, 64), "CD4", 0, True, False),
    (1, (20, 16, 64), "CD6", 0, False, False), (1, (12, 14, 16), "E8", 0, False, False),
    (0, (45, 64), "CD4", 0, False, True)])
def test_restart_is_bitwise(L, orc, lat, shape, scheme, coll, wall, nofused, monkeypatch):
    import torch
    p, rho0, solid = _case(L, orc, lat, shape, scheme, coll, wall)
    if nofused:
        monkeypatch.setenv("LBM_NO_FUSED", "1")
    probe = L.Simulation(p, rho0, solid=solid)
    variants = list(range(probe.num_variants))
    probe.close()
    other = np.full(rho0.shape, float(rho0.mean()))   # the loaded state replaces this one
    for v in variants:
        a = L.Simulation(p, rho0, solid=solid)
        a.set_variant(v)
        a.step(15)
        img_h = a.save_state()
        img_d = a.save_state(device=True)
        assert img_h.nbytes == 64 + 8 * (p.q + 1) * p.n
        assert np.array_equal(img_h, img_d.cpu().numpy())
        f_saved = a.populations()
        a.step(12)
        for img in (img_h, img_d):
            b = L.Simulation(p, other, solid=solid)
            b.set_variant(v)
            b.step(3)                       # some history of its own first
            b.load_state(img)
            assert b.steps_done == 15
            assert np.array_equal(b.populations(), f_saved)
            b.step(12)
            assert b.steps_done == 27
            assert np.array_equal(b.populations(), a.populations()), (v, type(img))
            assert np.array_equal(b.macros()[0], a.macros()[0])
            b.close()
        print(f"case restart lattice={lat} shape={shape} scheme={scheme} variant={v} {a.variant_name(v)!r}: bitwise",
              flush=True)
        a.close()
        torch.cuda.empty_cache()


def test_restart_refusals(L, orc):
    p, rho0, _ = _case(L, orc, 0, (40, 44), "CD4")
    a = L.Simulation(p, rho0)
    a.step(5)
    img = a.save_state()
    q, _, _ = _case(L, orc, 0, (40, 48), "CD4")
    b = L.Simulation(q, inputs.droplet((40, 48), 10, 4.0, *orc.maxwell(0.8)))
    with pytest.raises(L.LbmError) as e:
        b.load_state(img)
    assert e.value.code == L.LBM_EINVAL
    bad = img.copy()
    bad[0] ^= 0xFF
    with pytest.raises(L.LbmError) as e:
        a.load_state(bad)
    assert e.value.code == L.LBM_EINVAL
    # a failed load leaves the state as it was
    f = a.populations()
    with pytest.raises(L.LbmError):
        a.load_state(bad)
    assert np.array_equal(a.populations(), f) and a.steps_done == 5
    # a batch instance can be saved, not loaded
    bt = L.Batch([p], [rho0])
    bt.run(5, check_every=5, tol=0.0, chunk=5)
    view = bt.instance(0)
    vimg = view.save_state()
    assert vimg.nbytes == img.nbytes
    hdr = np.frombuffer(vimg[:64].tobytes(), np.int64)
    assert list(hdr[2:7]) == [L.D2Q9, 44, 40, 1, 5]
    with pytest.raises(L.LbmError) as e:
        view.load_state(img)
    assert e.value.code == L.LBM_ESTATE
