"""Learned initial condition: a small network, trained by the library's FP32
kernels on equilibrium droplet profiles produced by the batched sweep, proposes
the equilibrium radial density profile and replaces the tanh start of Eq 26.

Data: droplets (D2Q9) run by the batched kernel; from each, four rays (+x, -x,
+y, -y) from the centre give profiles rho(r); R_eq is where rho crosses the
mean of its centre and edge values (linear interpolation); samples are
(Tr, k, scheme id, r - R_eq) -> phi = (rho - rho_g^M)/(rho_l^M - rho_g^M) with
the Maxwell densities.  Training: mean-squared error, Adam, on the GPU kernels
(mlp_forward / mlp_loss_grad / mlp_backward / mlp_adam).  Use: the initial
field comes from mlp_field with R chosen by bisection so that the total mass
equals that of the tanh start; a non-finite or failed match falls back to tanh.
"""
from __future__ import annotations

import ctypes as C
import json
import os
import sys
import time

import numpy as np

from . import inputs, lbm

SCHEMES6 = [lbm.CD2, lbm.CD4, lbm.CD6, lbm.E4, lbm.E8, lbm.OCFDS4]
# feature scaling: (Tr - 0.75) / 0.15, (k - 0.175) / 0.05, (scheme - 2.5) / 1.7,
# distance / 10
NORM = np.array([0.75, 1 / 0.15, 0.175, 1 / 0.05, 2.5, 1 / 1.7, 10.0], dtype=np.float32)


def features(Tr, k, scheme):
    return np.array([(Tr - NORM[0]) * NORM[1], (k - NORM[2]) * NORM[3], (scheme - NORM[4]) * NORM[5]],
                    dtype=np.float32)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _progress(tag):
    def cb(done, status):
        log(f"{tag}: {done} steps, running {(status == 0).sum()}, converged {(status == 1).sum()}, "
            f"diverged {(status == 2).sum()}")
    return cb


class Net:
    """Network parameters and Adam moments on the device (torch float32)."""

    def __init__(self, seed: int = 0, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.P = int(lbm.lib().mlp_param_count())
        self.params = torch.from_numpy(self.init_params(seed)).to(self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.stream = torch.cuda.current_stream(self.device)

    @staticmethod
    def init_params(seed: int) -> np.ndarray:
        rng = np.random.default_rng(inputs.SEED_BASE + 1000 + seed)
        sizes = [4, 64, 64, 64, 1]
        parts = []
        for i in range(4):
            fi, fo = sizes[i], sizes[i + 1]
            lim = np.sqrt(6.0 / fi) * (0.5 if i == 3 else 1.0)
            parts.append(rng.uniform(-lim, lim, fo * fi))
            parts.append(np.zeros(fo))
        return np.concatenate(parts).astype(np.float32)

    def forward(self, X, acts=None):
        t = self.torch
        B = X.shape[0]
        y = t.empty(B, dtype=t.float32, device=self.device)
        lbm._check(lbm.lib().mlp_forward(_ptr(self.params), _ptr(X), B, _ptr(y),
                                         _ptr(acts) if acts is not None else None, C.c_void_p(self.stream.cuda_stream)))
        return y

    def grad(self, X, T):
        """(loss, gradient) of the mean-squared error on (X, T), all on the device."""
        t = self.torch
        B = X.shape[0]
        nb = (B + 63) // 64
        acts = t.empty(B * 192, dtype=t.float32, device=self.device)
        y = self.forward(X, acts)
        dy = t.empty(B, dtype=t.float32, device=self.device)
        lp = t.empty(nb, dtype=t.float32, device=self.device)
        g = t.empty(self.P, dtype=t.float32, device=self.device)
        gp = t.empty(nb * self.P, dtype=t.float32, device=self.device)
        s = C.c_void_p(self.stream.cuda_stream)
        lbm._check(lbm.lib().mlp_loss_grad(_ptr(y), _ptr(T), B, _ptr(dy), _ptr(lp), s))
        lbm._check(lbm.lib().mlp_backward(_ptr(self.params), _ptr(X), _ptr(acts), _ptr(dy), B, _ptr(g), _ptr(gp), s))
        return lp, g

    def adam(self, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        lbm._check(lbm.lib().mlp_adam(_ptr(self.params), _ptr(g), _ptr(self.m), _ptr(self.v), self.t, lr, b1, b2, eps,
                                      C.c_void_p(self.stream.cuda_stream)))

    def train(self, X, T, iters=3000, batch=4096, lr=2e-3, seed=0, log_every=500):
        """Minibatch Adam on device data X (n, 4), T (n,)."""
        t = self.torch
        rng = np.random.default_rng(inputs.SEED_BASE + 2000 + seed)
        n = X.shape[0]
        hist = []
        for it in range(1, iters + 1):
            idx = t.from_numpy(rng.integers(0, n, batch)).to(self.device)
            xb, tb = X.index_select(0, idx).contiguous(), T.index_select(0, idx).contiguous()
            lr_t = lr * (0.1 ** (it / iters))
            lp, g = self.grad(xb, tb)
            self.adam(g, lr=lr_t)
            if it % log_every == 0 or it == iters:
                hist.append((it, float(lp.sum().item()) / batch))
                log(f"train {it}/{iters} loss {hist[-1][1]:.3e}")
        return hist

    def field(self, p: lbm.Params, R, Tr, k, scheme, rho_g, rho_l, center=None):
        """Initial density of the whole grid (device float64 tensor)."""
        t = self.torch
        out = t.empty(p.n, dtype=t.float64, device=self.device)
        c = center or (p.nx // 2, p.ny // 2, p.nz // 2 if p.lattice == lbm.D3Q19 else 0)
        norm = (C.c_float * 7)(*NORM.tolist())
        feat = (C.c_float * 3)(*features(Tr, k, scheme).tolist())
        cp = p.c()
        lbm._check(lbm.lib().mlp_field(_ptr(self.params), norm, C.byref(cp), float(c[0]), float(c[1]), float(c[2]),
                                       float(R), feat, float(rho_g), float(rho_l), _ptr(out),
                                       C.c_void_p(self.stream.cuda_stream)))
        return out

    def state(self):
        return self.params.cpu().numpy()

    def load(self, arr):
        self.params.copy_(self.torch.from_numpy(np.asarray(arr, dtype=np.float32)).to(self.device))


def device_sum(x) -> float:
    import torch
    n = x.numel()
    scratch = torch.empty(int(lbm.lib().lbm_sum_scratch_bytes(n)) // 8 + 1, dtype=torch.float64, device=x.device)
    s = C.c_double()
    lbm._check(lbm.lib().lbm_sum(_ptr(x), n, _ptr(scratch), C.byref(s),
                                 C.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)))
    return s.value


def mass_matched_field(net: Net, p: lbm.Params, R0, Tr, k, scheme, rho_g, rho_l, target_mass, iters=60,
                       rel_tol=1e-10, noise=None):
    """Bisection on the radius so that the learned field has the target mass,
    then lbm_interface_mass for the residual the FP32 network leaves (only
    interface nodes change; the bulk densities stay as the network set them).
    noise (host array of p.n values, or None): the relative perturbation the
    tanh start carries (inputs.droplet with relative=True), applied to the
    field before the residual is taken, so that both starts carry the same one.
    Returns (rho0 device tensor, radius), or (None, R0) when the target is not
    bracketed or the mass still misses it by more than rel_tol."""
    lo, hi = 0.25 * R0, min(p.nx, p.ny) * 0.5
    f_lo = device_sum(net.field(p, lo, Tr, k, scheme, rho_g, rho_l)) - target_mass
    f_hi = device_sum(net.field(p, hi, Tr, k, scheme, rho_g, rho_l)) - target_mass
    if not (np.isfinite(f_lo) and np.isfinite(f_hi)) or f_lo > 0 or f_hi < 0:
        return None, R0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        fm = device_sum(net.field(p, mid, Tr, k, scheme, rho_g, rho_l)) - target_mass
        if fm < 0:
            lo = mid
        else:
            hi = mid
    R = 0.5 * (lo + hi)
    rho = net.field(p, R, Tr, k, scheme, rho_g, rho_l)
    import torch
    if noise is not None:
        # input preparation, on the host as in inputs.droplet
        rho = torch.from_numpy(rho.cpu().numpy() * (1.0 + np.asarray(noise, np.float64).reshape(-1))).to(rho.device)
    # the network evaluates in FP32, so the mass moves in small steps with R:
    # the library puts the last residual into the interface nodes
    scratch = torch.empty(int(lbm.lib().lbm_sum_scratch_bytes(rho.numel())) // 8 + 1, dtype=torch.float64,
                          device=rho.device)
    lbm._check(lbm.lib().lbm_interface_mass(_ptr(rho), rho.numel(), float(rho_g), float(rho_l), float(target_mass),
                                            _ptr(scratch), C.c_void_p(torch.cuda.current_stream(rho.device).cuda_stream)))
    if not abs(device_sum(rho) - target_mass) <= rel_tol * abs(target_mass):
        return None, R0
    return rho, R


# Under the SRT collision the second-order and isotropic schemes are stable
# only near the critical point; each scheme draws its temperature from the
# range where it runs.
STABLE_TR = {lbm.CD2: (0.9, 0.95), lbm.E4: (0.9, 0.95), lbm.E8: (0.9, 0.95)}


def droplet_set(n, seed, r_range=(12.0, 50.0), tr_range=(0.6, 0.9), k_range=(0.1, 0.25), lmax=256):
    rng = np.random.default_rng(inputs.SEED_BASE + 3000 + seed)
    out = []
    for i in range(n):
        R = float(rng.uniform(*r_range))
        lo = max(64, int(np.ceil((2 * R + 64) / 8.0)) * 8)
        L = int(rng.integers(lo // 8, max(lo, lmax) // 8 + 1)) * 8
        sch = SCHEMES6[int(rng.integers(0, 6))]
        tr = STABLE_TR.get(sch, tr_range)
        out.append(dict(L=L, R=R, Tr=float(rng.uniform(*tr)), k=float(rng.uniform(*k_range)),
                        scheme=sch, instance_id=10000 + 1000 * seed + i))
    return out


def _tanh_batch(specs, width=10.0, kappa=0.004):
    ps, rs = [], []
    for d in specs:
        g, l = lbm.coexistence(d["Tr"])
        ps.append(lbm.Params(lattice=lbm.D2Q9, nx=d["L"], ny=d["L"], Tr=d["Tr"], k=d["k"], kappa=kappa,
                             scheme=d["scheme"]))
        rs.append(inputs.droplet((d["L"], d["L"]), d["R"], width, g, l, instance_id=d["instance_id"], relative=True))
    return ps, rs


def profiles(batch_views, specs):
    """Samples (features..., distance) -> phi from the rays of each droplet."""
    X, T = [], []
    for v, d in zip(batch_views, specs):
        r = v.macros()[0]
        L = d["L"]
        c = L // 2
        g, l = lbm.coexistence(d["Tr"])
        f = features(d["Tr"], d["k"], d["scheme"])
        rays = [r[c, c:], r[c, c::-1], r[c:, c], r[c::-1, c]]
        for ray in rays:
            ray = np.asarray(ray[: L // 2])
            # keep only droplets that are still droplets: liquid at the centre,
            # gas at the edge (a small droplet can dissolve into the vapour)
            phi0, phi1 = (ray[0] - g) / (l - g), (ray[-1] - g) / (l - g)
            if not (phi0 > 0.8 and phi1 < 0.2):
                continue
            mid = 0.5 * (ray[0] + ray[-1])
            below = np.nonzero(ray < mid)[0]
            if below.size == 0 or below[0] < 4:
                continue
            j = below[0]
            Req = (j - 1) + (ray[j - 1] - mid) / (ray[j - 1] - ray[j])
            dist = (np.arange(ray.size) - Req) / NORM[6]
            phi = (ray - g) / (l - g)
            X.append(np.column_stack([np.tile(f, (ray.size, 1)), dist]))
            T.append(phi)
    return np.concatenate(X).astype(np.float32), np.concatenate(T).astype(np.float32)


def make_dataset(n_batches=5, per_batch=96, steps=6000, seed=0):
    X, T, nprof, status = [], [], 0, []
    for bi in range(n_batches):
        specs = droplet_set(per_batch, seed * 100 + bi, r_range=(12.0, 50.0), tr_range=(0.6, 0.95), lmax=160)
        ps, rs = _tanh_batch(specs)
        b = lbm.Batch(ps, rs)
        b.set_form(lbm.BATCH_PHASES)
        st, _, _ = b.run(steps, check_every=100, tol=1e-10, chunk=2000, progress=_progress(f"data batch {bi}"))
        ok = [i for i in range(len(specs)) if st[i] != lbm.DIVERGED]
        status += list(st)
        x, t = profiles([b.instance(i) for i in ok], [specs[i] for i in ok])
        X.append(x); T.append(t)
        nprof += 4 * len(ok)
        b.close()
    return np.concatenate(X), np.concatenate(T), nprof, status


def evaluate(net: Net, n=64, seed=7, max_steps=30000, check_every=100, tol=1e-10, chunk=2000):
    """Held-out droplets from the tanh start and from the learned start (same
    mass); steps to |U(t) - U(t-100)| < tol and the final state of both."""
    import torch
    specs = droplet_set(n, 50 + seed)
    ps, rs = _tanh_batch(specs)
    learned, fallback = [], 0
    log(f"eval: building {len(specs)} learned initial states")
    for p, r, d in zip(ps, rs, specs):
        g, l = lbm.coexistence(d["Tr"])
        rho, _ = mass_matched_field(net, p, d["R"], d["Tr"], d["k"], d["scheme"], g, l, float(r.sum()),
                                    noise=inputs.noise(r.shape, 1e-6, d["instance_id"]))
        if rho is None or not bool(torch.isfinite(rho).all()):
            fallback += 1
            learned.append(r)
        else:
            learned.append(rho.cpu().numpy().reshape(r.shape))
    out = {}
    for name, rhos in (("tanh", rs), ("learned", learned)):
        b = lbm.Batch(ps, rhos)
        b.set_form(lbm.BATCH_PHASES)
        t0 = time.perf_counter()
        st, steps, U = b.run(max_steps, check_every=check_every, tol=tol, chunk=chunk, progress=_progress(name))
        wall = time.perf_counter() - t0
        dens = []
        for i, d in enumerate(specs):
            if st[i] == lbm.DIVERGED:
                dens.append((np.nan, np.nan))
                continue
            rr = b.instance(i).macros()[0]
            dens.append((float(rr[d["L"] // 2, d["L"] // 2]), float(rr[0, 0])))
        out[name] = dict(status=st.tolist(), steps=steps.tolist(), U=U.tolist(), dens=dens, wall_s=wall)
        b.close()
    both = [i for i in range(n) if out["tanh"]["status"][i] == lbm.CONVERGED and
            out["learned"]["status"][i] == lbm.CONVERGED]
    ratio = [out["learned"]["steps"][i] / out["tanh"]["steps"][i] for i in both]
    du = [abs(out["learned"]["U"][i] - out["tanh"]["U"][i]) / max(abs(out["tanh"]["U"][i]), 1e-300) for i in both]
    dl = [abs(out["learned"]["dens"][i][0] - out["tanh"]["dens"][i][0]) / out["tanh"]["dens"][i][0] for i in both]
    dg = [abs(out["learned"]["dens"][i][1] - out["tanh"]["dens"][i][1]) / out["tanh"]["dens"][i][1] for i in both]
    summary = dict(n=n, fallback=fallback, both_converged=len(both),
                   steps_ratio_median=float(np.median(ratio)) if ratio else None,
                   steps_ratio_quartiles=[float(np.percentile(ratio, q)) for q in (25, 75)] if ratio else None,
                   learned_fewer_steps=int(sum(1 for x in ratio if x < 1)),
                   U_reldiff_max=float(max(du)) if du else None, rho_l_reldiff_max=float(max(dl)) if dl else None,
                   rho_g_reldiff_max=float(max(dg)) if dg else None,
                   tanh_counts={k: out["tanh"]["status"].count(v) for k, v in
                                (("running", 0), ("converged", 1), ("diverged", 2))},
                   learned_counts={k: out["learned"]["status"].count(v) for k, v in
                                   (("running", 0), ("converged", 1), ("diverged", 2))})
    return summary, out


NET_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "learned_net.npy")


def gain(net: Net = None, n: int = 16, seed: int = 60, lmax: int = 128, tol: float = 1e-12,
         max_steps: int = 300000, check_every: int = 100, chunk: int = 20000):
    """What the learned start gains over the tanh start (Eq 26, width 10):
    n held-out D2Q9 droplets (a seed disjoint from the training and earlier
    evaluation sets; each scheme in the temperature range where it runs under
    SRT) from both starts, mass-matched, run by the batched kernel until
    |U(t) - U(t - check_every)| < tol.  Droplets that end as droplets from
    both starts (centre density above 1.5 x the corner's) are compared: the
    ratio of steps, the final U and the centre (rho_l) and corner (rho_g)
    densities.  Returns (summary, rows)."""
    import torch
    if net is None:
        net = Net(0)
        net.load(np.load(NET_PATH))
    specs = droplet_set(n, seed=seed, lmax=lmax)
    ps, rs = _tanh_batch(specs)
    starts, fallback = [], 0
    for p, r, d in zip(ps, rs, specs):
        g, l = lbm.coexistence(d["Tr"])
        rho, _ = mass_matched_field(net, p, d["R"], d["Tr"], d["k"], d["scheme"], g, l, float(r.sum()),
                                    noise=inputs.noise(r.shape, 1e-6, d["instance_id"]))
        if rho is None or not bool(torch.isfinite(rho).all()):
            fallback += 1
            starts.append(r)
        else:
            starts.append(rho.cpu().numpy().reshape(r.shape))
    res = {}
    for name, rhos in (("tanh", rs), ("learned", starts)):
        b = lbm.Batch(ps, rhos)
        # one launch per phase: bitwise the states of the persistent kernel,
        # in less time on these sets
        b.set_form(lbm.BATCH_PHASES)
        t0 = time.perf_counter()
        st, steps, U = b.run(max_steps, check_every=check_every, tol=tol, chunk=chunk)
        wall = time.perf_counter() - t0
        dens = []
        for i, d in enumerate(specs):
            rr = b.instance(i).macros()[0]
            dens.append((float(rr[d["L"] // 2, d["L"] // 2]), float(rr[0, 0])))
        res[name] = (st, steps, U, dens, wall, b.launch_mode)
        b.close()
    return gain_summary(specs, fallback, res["tanh"], res["learned"])


def gain_summary(specs, fallback, t, lrn):
    """Rows and summary of the learned-vs-tanh comparison (host logic).
    t and lrn are the two runs' (status, steps, U, [(centre, corner) density],
    wall seconds, launch mode), one entry per droplet of specs.  A droplet is
    compared when both runs met the criterion and both still hold a droplet
    (centre density above 1.5 x the corner's); the steps saved are counted over
    every droplet whose two runs met the criterion, since a run stopped by the
    cap would count its cap as its steps."""
    n = len(specs)
    rows = []
    for i, d in enumerate(specs):
        row = dict(L=d["L"], R=d["R"], scheme=int(d["scheme"]), Tr=d["Tr"], k=d["k"],
                   status=(int(t[0][i]), int(lrn[0][i])), steps=(int(t[1][i]), int(lrn[1][i])))
        ok = t[0][i] == lbm.CONVERGED and lrn[0][i] == lbm.CONVERGED
        if ok and t[3][i][0] > 1.5 * t[3][i][1] and lrn[3][i][0] > 1.5 * lrn[3][i][1]:
            row.update(ratio=lrn[1][i] / t[1][i], dU=abs(lrn[2][i] - t[2][i]) / abs(t[2][i]),
                       dl=abs(lrn[3][i][0] - t[3][i][0]) / t[3][i][0],
                       dg=abs(lrn[3][i][1] - t[3][i][1]) / t[3][i][1])
        rows.append(row)
    cmp_ = [r for r in rows if "ratio" in r]
    ratio = np.array([r["ratio"] for r in cmp_])
    dU = np.array([r["dU"] for r in cmp_])
    both = [i for i in range(n) if t[0][i] == lbm.CONVERGED and lrn[0][i] == lbm.CONVERGED]
    st_t = sum(int(t[1][i]) for i in both)
    st_l = sum(int(lrn[1][i]) for i in both)
    summary = dict(
        droplets=n, fallback=fallback, compared=len(cmp_),
        steps_ratio_median=float(np.median(ratio)) if cmp_ else None,
        learned_fewer_steps=int((ratio < 1).sum()),
        steps_saved_total=float(1 - st_l / st_t) if st_t > 0 else None,
        both_converged=len(both),
        not_converged={"tanh": int(sum(int(x) != lbm.CONVERGED for x in t[0])),
                       "learned": int(sum(int(x) != lbm.CONVERGED for x in lrn[0]))},
        U_reldiff_median=float(np.median(dU)) if cmp_ else None,
        U_reldiff_max=float(dU.max()) if cmp_ else None,
        U_within_1e6=int((dU <= 1e-6).sum()),
        rho_l_reldiff_max=max((r["dl"] for r in cmp_), default=None),
        rho_g_reldiff_max=max((r["dg"] for r in cmp_), default=None),
        wall_s={"tanh": round(t[4], 2), "learned": round(lrn[4], 2)},
        launch={"tanh": t[5], "learned": lrn[5]})
    return summary, rows


def droplet_set_3d(n, seed, r_frac=(0.22, 0.32), tr_range=(0.65, 0.85), k_range=(0.1, 0.25), sides=(96, 128)):
    """Seeded 3D droplets (D3Q19, L^3 periodic) for the learned start in 3D.
    The radius is a fraction of the box: smaller droplets evaporate into the
    vapour of a periodic box (more readily in 3D than in 2D)."""
    rng = np.random.default_rng(inputs.SEED_BASE + 5000 + seed)
    out = []
    for i in range(n):
        L = int(sides[int(rng.integers(0, len(sides)))])
        R = float(rng.uniform(*r_frac)) * L
        sch = SCHEMES6[int(rng.integers(0, 6))]
        tr = STABLE_TR.get(sch, tr_range)
        out.append(dict(L=L, R=R, Tr=float(rng.uniform(*tr)), k=float(rng.uniform(*k_range)),
                        scheme=sch, instance_id=20000 + 1000 * seed + i))
    return out


def big_droplet(net: Net, scheme: int, L: int = 384, R: float = 80.0, Tr: float = 0.8, k: float = 0.1,
                max_steps: int = 40000, check_every: int = 100, tol: float = 1e-10, report_every: int = 2000,
                starts=("tanh", "learned")):
    """The config-5 geometry (D3Q19 L^3 periodic, droplet of radius R at the
    centre) from the tanh start of Eq 26 (width 10) and from the learned start
    (same mass), each run on a plain context until |U(t) - U(t - 100)| < tol
    or max_steps (starts: which of the two to run).  Returns one row per
    start: status, steps, U, rho_l at the centre, rho_g at the corner, MLUPS
    of the stepping, and the U history."""
    import torch
    g, l = lbm.coexistence(Tr)
    p = lbm.Params(lattice=lbm.D3Q19, nx=L, ny=L, nz=L, Tr=Tr, k=k, kappa=0.004, scheme=scheme)
    r_t = inputs.droplet((L, L, L), R, 10.0, g, l, instance_id=30000 + scheme, relative=True)
    rho, _ = mass_matched_field(net, p, R, Tr, k, scheme, g, l, float(r_t.sum()),
                                noise=inputs.noise(r_t.shape, 1e-6, 30000 + scheme))
    rows = {}
    for name, r0 in (("tanh", r_t), ("learned", rho if rho is not None else r_t)):
        if name not in starts:
            continue
        sim = lbm.Simulation(p, torch.from_numpy(r0.reshape(-1)).cuda() if isinstance(r0, np.ndarray) else r0)
        # the fastest collide on 256^3 and 384^3 (no tuner: it would advance the state)
        names = [sim.variant_name(v) for v in range(sim.num_variants)]
        if "tile 64x16 z64" in names:
            sim.set_variant(names.index("tile 64x16 z64"))
        steps, U_prev, status, hist, t_step = 0, None, lbm.RUNNING, [], 0.0
        while True:
            U = float(sim.spurious_max()[0])
            if steps % report_every == 0:
                hist.append((steps, U))
                log(f"big droplet {L}^3 scheme {scheme} {name}: step {steps} U {U:.6e}")
            if not np.isfinite(U) or U > 3 ** -0.5:
                status = lbm.DIVERGED
                break
            if U_prev is not None and abs(U - U_prev) < tol:
                status = lbm.CONVERGED
                break
            if steps >= max_steps:
                break
            U_prev = U
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(check_every)
            torch.cuda.synchronize()
            t_step += time.perf_counter() - t0
            steps += check_every
        r = sim.macros()[0] if status != lbm.DIVERGED else None
        rows[name] = dict(status=int(status), steps=steps, U=U, fallback=rho is None and name == "learned",
                          rho_l=float(r[L // 2, L // 2, L // 2]) if r is not None else None,
                          rho_g=float(r[0, 0, 0]) if r is not None else None,
                          mlups=p.n * steps / t_step / 1e6 if t_step > 0 else None, history=hist)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    return dict(L=L, R=R, Tr=Tr, k=k, scheme=scheme, rho_g_maxwell=g, rho_l_maxwell=l, runs=rows)


def run_to_equilibrium(p: lbm.Params, rho0, max_steps, check_every=100, tol=1e-10):
    """One plain context from rho0 under the convergence rule of the batched
    sweep: U = max|v| is taken every check_every steps before stepping on;
    converged at the first check t > 0 with |U(t) - U(t - check_every)| < tol,
    diverged on a non-finite state or U above the sound speed.
    Returns (status, steps, U, rho_l at the centre, rho_g at the corner)."""
    sim = lbm.Simulation(p, rho0)
    steps, U_prev, status, U = 0, None, lbm.RUNNING, float("nan")
    while True:
        U = float(sim.spurious_max()[0])
        if not np.isfinite(U) or U > 3 ** -0.5:
            status = lbm.DIVERGED
            break
        if U_prev is not None and abs(U - U_prev) < tol:
            status = lbm.CONVERGED
            break
        if steps >= max_steps:
            break
        U_prev = U
        sim.step(check_every)
        steps += check_every
    if status == lbm.DIVERGED:
        sim.close()
        return status, steps, U, float("nan"), float("nan")
    r = sim.macros()[0]
    sim.close()
    c = tuple(s // 2 for s in r.shape)
    return status, steps, U, float(r[c]), float(r[(0,) * r.ndim])


def evaluate_3d(net: Net, n=8, seed=7, max_steps=60000, check_every=100, tol=1e-10):
    """3D droplets started from tanh (Eq 26, W = 10) and from the learned
    profile (trained on 2D droplets; same mass), each run to equilibrium."""
    import torch
    specs = droplet_set_3d(n, seed)
    rows, fallback = [], 0
    for i, d in enumerate(specs):
        L = d["L"]
        g, l = lbm.coexistence(d["Tr"])
        p = lbm.Params(lattice=lbm.D3Q19, nx=L, ny=L, nz=L, Tr=d["Tr"], k=d["k"], kappa=0.004, scheme=d["scheme"])
        r_t = inputs.droplet((L, L, L), d["R"], 10.0, g, l, instance_id=d["instance_id"], relative=True)
        rho, _ = mass_matched_field(net, p, d["R"], d["Tr"], d["k"], d["scheme"], g, l, float(r_t.sum()),
                                    noise=inputs.noise(r_t.shape, 1e-6, d["instance_id"]))
        if rho is None or not bool(torch.isfinite(rho).all()):
            fallback += 1
            r_l = r_t
        else:
            r_l = rho.cpu().numpy().reshape(r_t.shape)
        row = dict(spec=d)
        for name, r0 in (("tanh", r_t), ("learned", r_l)):
            st, steps, U, rl, rg = run_to_equilibrium(p, r0, max_steps, check_every, tol)
            row[name] = dict(status=int(st), steps=int(steps), U=U, rho_l=rl, rho_g=rg)
        log(f"eval3d {i + 1}/{n}: L={L} R={d['R']:.1f} scheme={d['scheme']} Tr={d['Tr']:.3f} "
            f"tanh {row['tanh']['status']}/{row['tanh']['steps']} learned {row['learned']['status']}/"
            f"{row['learned']['steps']}")
        rows.append(row)
    both = [r for r in rows if r["tanh"]["status"] == lbm.CONVERGED and r["learned"]["status"] == lbm.CONVERGED]
    ratio = [r["learned"]["steps"] / r["tanh"]["steps"] for r in both]
    du = [abs(r["learned"]["U"] - r["tanh"]["U"]) / abs(r["tanh"]["U"]) for r in both]
    summary = dict(n=n, fallback=fallback, both_converged=len(both),
                   dissolved=int(sum(1 for r in rows if r["tanh"]["status"] == lbm.CONVERGED
                                     and r["tanh"]["rho_l"] < 1.5 * r["tanh"]["rho_g"])),
                   steps_ratio=ratio, steps_ratio_median=float(np.median(ratio)) if ratio else None,
                   learned_fewer_steps=int(sum(1 for x in ratio if x < 1)),
                   U_reldiff=du,
                   rho_l_reldiff_max=max((abs(r["learned"]["rho_l"] - r["tanh"]["rho_l"]) / r["tanh"]["rho_l"]
                                          for r in both), default=None),
                   rho_g_reldiff_max=max((abs(r["learned"]["rho_g"] - r["tanh"]["rho_g"]) / r["tanh"]["rho_g"]
                                          for r in both), default=None))
    return summary, rows


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--batches", type=int, default=5)
    ap.add_argument("--data-steps", type=int, default=6000)
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--eval", type=int, default=64)
    ap.add_argument("--max-steps", type=int, default=30000)
    ap.add_argument("--save", default="")
    ap.add_argument("--dump", default="", help="directory for the dataset and per-instance results")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--load", default="", help="parameters saved by --save: skip the dataset and the training")
    ap.add_argument("--eval-seed", type=int, default=7, help="seed of the held-out droplet set")
    ap.add_argument("--eval3d", type=int, default=0,
                    help="also this many 3D (D3Q19) droplets, tanh vs learned start, each run to equilibrium")
    ap.add_argument("--max-steps-3d", type=int, default=60000)
    ap.add_argument("--tol", type=float, default=1e-10, help="convergence: |U(t) - U(t - 100)| < tol")
    ap.add_argument("--big", default="", help="comma-separated schemes: the config-5 droplet (D3Q19 384^3, R 80) "
                                              "at --big-Tr from the tanh and the learned start")
    ap.add_argument("--big-Tr", type=float, default=0.8)
    ap.add_argument("--big-n", type=int, default=384)
    ap.add_argument("--big-start", default="both", choices=["both", "tanh", "learned"],
                    help="run the config-5 droplet from this start only")
    a = ap.parse_args()
    if a.big:
        net = Net(0)
        net.load(np.load(a.load))
        starts = ("tanh", "learned") if a.big_start == "both" else (a.big_start,)
        res = [big_droplet(net, lbm.SCHEMES[sname], L=a.big_n, R=80.0 * a.big_n / 384, Tr=a.big_Tr,
                           max_steps=a.max_steps_3d, tol=a.tol, starts=starts) for sname in a.big.split(",")]
        print(json.dumps(res))
        return
    import torch
    t0 = time.perf_counter()
    if a.dump:
        os.makedirs(a.dump, exist_ok=True)
    net = Net(0)
    if a.load:
        net.load(np.load(a.load))
        nprof, X, st, hist = 0, np.zeros((0, 4), np.float32), [], []
        t1 = t2 = time.perf_counter()
    else:
        X, T, nprof, st = make_dataset(a.batches, steps=a.data_steps)
        t1 = time.perf_counter()
        if a.dump:
            np.save(os.path.join(a.dump, "X.npy"), X)
            np.save(os.path.join(a.dump, "T.npy"), T)
        hist = net.train(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), iters=a.iters, lr=a.lr,
                         batch=a.batch)
        t2 = time.perf_counter()
    summary, full = (evaluate(net, n=a.eval, seed=a.eval_seed, max_steps=a.max_steps, tol=a.tol) if a.eval > 0
                     else (None, None))
    if a.dump and full is not None:
        json.dump(full, open(os.path.join(a.dump, "eval_full.json"), "w"))
    summary3d = None
    if a.eval3d > 0:
        summary3d, rows3d = evaluate_3d(net, n=a.eval3d, seed=a.eval_seed, max_steps=a.max_steps_3d, tol=a.tol)
        if a.dump:
            json.dump(rows3d, open(os.path.join(a.dump, "eval3d_full.json"), "w"))
    t3 = time.perf_counter()
    if a.save:
        np.save(a.save, net.state())
    print(json.dumps(dict(profiles=nprof, samples=int(X.shape[0]), data_diverged=int(sum(1 for s in st if s == 2)),
                          train_history=hist, eval=summary, eval3d=summary3d,
                          seconds=dict(data=t1 - t0, train=t2 - t1, eval=t3 - t2))))


if __name__ == "__main__":
    main()
