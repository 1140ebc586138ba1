"""FP32 network kernels of the learned initialiser against the FP64 CPU
reference (forward, backpropagated gradients, Adam, field inference)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_09186_amd import lbm, learned
    from oracle import mlp
    lbm.lib()
    return torch, lbm, learned, mlp


def _data(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, 4)).astype(np.float32)
    T = rng.uniform(0, 1, B).astype(np.float32)
    return X, T


def test_forward_matches_reference(env):
    torch, lbm, learned, mlp = env
    net = learned.Net(1)
    theta = net.state().astype(np.float64)
    X, _ = _data(1000, 0)
    y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    yr, _ = mlp.forward(theta, X.astype(np.float64))
    assert np.abs(y - yr).max() <= 1e-5 * (1 + np.abs(yr).max())


@pytest.mark.parametrize("B", [64, 200, 4096])
def test_gradient_matches_fp64_backprop(env, B):
    torch, lbm, learned, mlp = env
    net = learned.Net(2)
    theta = net.state().astype(np.float64)
    X, T = _data(B, B)
    lp, g = net.grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    g = g.cpu().numpy().astype(np.float64)
    gr = mlp.grad(theta, X.astype(np.float64), T.astype(np.float64))
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    # per-layer norms too (a wrong small layer would hide in the total)
    offs = [0, 256, 320, 4416, 4480, 8576, 8640, 8704, 8705]
    for a, b in zip(offs[:-1], offs[1:]):
        assert np.linalg.norm(g[a:b] - gr[a:b]) <= 1e-4 * np.linalg.norm(gr[a:b]) + 1e-7, (a, b)
    assert float(lp.sum().item()) / B == pytest.approx(mlp.loss(theta, X.astype(np.float64), T.astype(np.float64)),
                                                       rel=1e-5)
    # deterministic reduction
    _, g2 = net.grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    assert np.array_equal(g2.cpu().numpy(), g.astype(np.float32))


def test_adam_step(env):
    torch, lbm, learned, mlp = env
    net = learned.Net(3)
    p0 = net.state().astype(np.float64)
    rng = np.random.default_rng(5)
    m = np.zeros_like(p0); v = np.zeros_like(p0); p = p0.copy()
    for step in range(1, 4):
        g = rng.standard_normal(p0.size).astype(np.float32)
        net.adam(torch.from_numpy(g).cuda(), lr=1e-2)
        gd = g.astype(np.float64)
        m = 0.9 * m + 0.1 * gd; v = 0.999 * v + 0.001 * gd * gd
        p = p - 1e-2 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
    assert np.abs(net.state() - p).max() < 1e-5


def test_field_inference_matches_reference(env):
    torch, lbm, learned, mlp = env
    net = learned.Net(4)
    theta = net.state().astype(np.float64)
    p = lbm.Params(lattice=lbm.D2Q9, nx=40, ny=30, Tr=0.8, k=0.2, scheme=lbm.CD6)
    g, l = 0.2, 7.2
    rho = net.field(p, 9.5, 0.8, 0.2, lbm.CD6, g, l).cpu().numpy().reshape(30, 40)
    f = learned.features(0.8, 0.2, lbm.CD6)
    ys, xs = np.mgrid[0:30, 0:40]
    d = (np.sqrt((xs - 20.0) ** 2 + (ys - 15.0) ** 2) - 9.5) / learned.NORM[6]
    X = np.column_stack([np.tile(f, (d.size, 1)), d.ravel()]).astype(np.float32)
    y, _ = mlp.forward(theta, X.astype(np.float64))
    ref = g + np.clip(y, 0, 1) * (l - g)
    assert np.abs(rho.ravel() - ref).max() < 1e-4


def test_field_inference_3d_matches_reference(env):
    """The same network sets the density of a 3D (D3Q19) droplet, by the
    Euclidean distance from the centre node (nx/2, ny/2, nz/2)."""
    torch, lbm, learned, mlp = env
    net = learned.Net(5)
    theta = net.state().astype(np.float64)
    p = lbm.Params(lattice=lbm.D3Q19, nx=20, ny=18, nz=16, Tr=0.75, k=0.15, scheme=lbm.OCFDS4)
    g, l = 0.1, 8.0
    rho = net.field(p, 6.3, 0.75, 0.15, lbm.OCFDS4, g, l).cpu().numpy().reshape(16, 18, 20)
    f = learned.features(0.75, 0.15, lbm.OCFDS4)
    zs, ys, xs = np.mgrid[0:16, 0:18, 0:20]
    d = (np.sqrt((xs - 10.0) ** 2 + (ys - 9.0) ** 2 + (zs - 8.0) ** 2) - 6.3) / learned.NORM[6]
    X = np.column_stack([np.tile(f, (d.size, 1)), d.ravel()]).astype(np.float32)
    y, _ = mlp.forward(theta, X.astype(np.float64))
    ref = g + np.clip(y, 0, 1) * (l - g)
    assert np.abs(rho.ravel() - ref).max() < 1e-4


def test_training_reduces_loss(env):
    torch, lbm, learned, mlp = env
    rng = np.random.default_rng(9)
    n = 20000
    Tr = rng.uniform(0.6, 0.95, n); k = rng.uniform(0.1, 0.25, n); s = rng.integers(0, 6, n)
    d = rng.uniform(-3, 3, n)
    width = 0.5 + 2.0 * (0.95 - Tr)                    # a smooth synthetic target family
    t = 0.5 - 0.5 * np.tanh(2.0 * d / width)
    X = np.column_stack([(Tr - 0.75) / 0.15, (k - 0.175) / 0.05, (s - 2.5) / 1.7, d]).astype(np.float32)
    net = learned.Net(0)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(t.astype(np.float32)).cuda()
    l0 = float(net.grad(Xd, Td)[0].sum().item()) / n
    hist = net.train(Xd, Td, iters=600, batch=2048, lr=3e-3, log_every=100)
    l1 = float(net.grad(Xd, Td)[0].sum().item()) / n
    assert l1 < 0.02 * l0, (l0, l1, hist)


@pytest.mark.parametrize("n", [1, 255, 256, 257, 100003, 3 * 2 ** 20 + 7])
def test_device_sum_is_accurate_and_repeatable(env, n):
    """lbm_sum (the mass of the learned start's bisection): a fixed-order tree,
    so two calls give the same bits; against math.fsum of the same doubles it
    is within the error bound of a pairwise sum of positive terms."""
    import math
    torch, lbm, learned, mlp = env
    rng = np.random.default_rng(n)
    x = rng.uniform(0.01, 10.0, n)
    t = torch.from_numpy(x).cuda()
    a, b = learned.device_sum(t), learned.device_sum(t)
    assert a == b
    exact = math.fsum(x)
    assert abs(a - exact) <= 4 * math.log2(n + 1) * 2.0 ** -53 * exact + 1e-300


def test_shipped_network_gives_a_droplet_profile(env):
    """The trained parameters shipped with the package: on a 2D droplet at
    T_r = 0.8 the field is liquid at the centre and gas far away, monotone
    along a ray, with its mid density within a node and a half of R."""
    import os
    torch, lbm, learned, mlp = env
    path = os.path.join(os.path.dirname(learned.__file__), "learned_net.npy")
    net = learned.Net(0)
    net.load(np.load(path))
    assert net.state().shape == (8705,)
    g, l = lbm.coexistence(0.8)
    p = lbm.Params(lattice=lbm.D2Q9, nx=96, ny=96, Tr=0.8, k=0.16, kappa=0.004, scheme=lbm.CD6)
    R = 24.0
    rho = net.field(p, R, 0.8, 0.16, lbm.CD6, g, l).cpu().numpy().reshape(96, 96)
    ray = rho[48, 48:]
    assert abs(ray[0] - l) < 0.05 * l and abs(ray[-1] - g) < 0.1 * (l - g)
    assert np.all(np.diff(ray) <= 1e-9 * l)
    mid = 0.5 * (l + g)
    j = int(np.nonzero(ray < mid)[0][0])
    r_mid = (j - 1) + (ray[j - 1] - mid) / (ray[j - 1] - ray[j])
    assert abs(r_mid - R) < 1.5, r_mid


def test_interface_mass_moves_only_the_interface(env):
    """lbm_interface_mass: the total reaches the target to rounding, nodes on
    either plateau keep their value bit for bit, interface nodes change in
    proportion to phi (1 - phi), and a second call on the same input gives
    the same field (fixed summation order)."""
    import ctypes as C
    from paper_2205_09186_amd import inputs
    torch, lbm, learned, mlp = env
    g, l = 0.197079412818, 7.20404871599
    r0 = inputs.droplet((150, 130), 40.0, 10.0, g, l, amplitude=0.0)
    # plateaus exactly at the coexistence values, a tanh interface between
    r0[r0 < g + 1e-3 * (l - g)] = g
    r0[r0 > l - 1e-3 * (l - g)] = l
    h = r0.reshape(-1)
    target = float(h.sum()) * (1 + 3e-7)
    outs = []
    for _ in range(2):
        d = torch.from_numpy(h.copy()).cuda()
        scratch = torch.empty(int(lbm.lib().lbm_sum_scratch_bytes(d.numel())) // 8 + 1, dtype=torch.float64,
                              device="cuda")
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        lbm._check(lbm.lib().lbm_interface_mass(C.c_void_p(d.data_ptr()), d.numel(), g, l, target,
                                                C.c_void_p(scratch.data_ptr()), st))
        outs.append(d.cpu().numpy())
    a, b = outs
    assert np.array_equal(a, b)
    assert abs(learned.device_sum(torch.from_numpy(a).cuda()) - target) <= 1e-13 * target
    phi = np.clip((h - g) / (l - g), 0.0, 1.0)
    w = phi * (1 - phi)
    flat = w == 0.0
    assert flat.sum() > h.size // 2 and np.array_equal(a[flat], h[flat])
    # a - h = c w with one constant c, to the rounding of the sum r + c w
    c = np.median((a - h)[~flat] / w[~flat])
    assert c > 0
    assert np.abs((a - h) - c * w).max() <= 4 * np.spacing(l)
    # bad arguments are refused before any launch
    assert lbm.lib().lbm_interface_mass(C.c_void_p(d.data_ptr()), d.numel(), l, g, target,
                                        C.c_void_p(scratch.data_ptr()), st) == lbm.LBM_EINVAL
