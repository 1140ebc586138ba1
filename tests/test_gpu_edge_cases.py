"""Degenerate cases through the C-ABI: no steps (the state is left as it is,
for a context and a batch), and the smallest periodic grids, whose stencils
wrap around an axis more than once (4 x 4 with CD6 and OCFDS4, 4 x 4 x 4 with
CD6, E8 and OCFDS4, 4 rows of 64 with CD4), on a smoothly perturbed gas,
against the oracle."""
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


def test_zero_steps_leave_the_state(L, orc):
    g, l = orc.maxwell(0.8)
    rho0 = inputs.droplet((24, 28), 6, 4.0, g, l)
    p = L.Params(lattice=L.D2Q9, nx=28, ny=24, Tr=0.8, k=0.16, kappa=0.004, scheme=L.CD4)
    s = L.Simulation(p, rho0)
    s.step(3)
    f = s.populations()
    s.step(0)
    assert s.steps_done == 3 and np.array_equal(s.populations(), f)
    b = L.Batch([p], [rho0])
    st, steps, _ = b.run(0, check_every=10, tol=0.0, chunk=10)
    assert list(st) == [L.RUNNING] and list(steps) == [0]
    st, steps, _ = b.run(3, check_every=10, tol=0.0, chunk=10)
    assert list(steps) == [3] and np.abs(b.instance(0).populations() - f).max() < 1e-11


@pytest.mark.parametrize("lat,shape,scheme", [(0, (4, 4), "CD6"), (0, (4, 4), "OCFDS4"), (1, (4, 4, 4), "CD6"),
                                              (1, (4, 4, 4), "E8"), (1, (4, 4, 4), "OCFDS4"), (0, (4, 64), "CD4")])
def test_smallest_grids_against_oracle(L, orc, lat, shape, scheme):
    g, l = orc.maxwell(0.9)
    # the gas density with a smooth periodic perturbation along every axis
    axes = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    pert = np.ones(shape)
    for a, n in zip(axes, shape):
        pert *= np.cos(2 * np.pi * a / n + 0.3)
    rho0 = g * (1.0 + 0.05 * pert)
    nz, ny, nx = ((1,) + shape) if lat == 0 else shape
    kw = dict(lattice=lat, nx=nx, ny=ny, nz=nz, Tr=0.9, k=0.16, kappa=0.004, scheme=L.SCHEMES[scheme])
    s = L.Simulation(L.Params(**kw), rho0)
    s.step(5)
    o = orc.Sim(orc.Params(**kw), rho0)
    o.step(5)
    got, ref = s.macros(), o.macros()
    d = max(np.abs(a - b).max() for a, b in zip(got, ref) if a is not None)
    print(f"case smallest grid lattice={lat} shape={shape} scheme={scheme}: max|diff| = {d:.2e}", flush=True)
    assert d <= 1e-11, d
