"""Diagnostic studies of Sec 3.1-3.2 built on the library's entry points.

* Flat interface (Sec 3.1, Eq 29).  For a flat interface in equilibrium the
  chemical potential is uniform, mu_hat = k^2 psi'(rho) - kappa_hat rho'' =
  k^2 mu_M, and a first integral gives
      kappa_hat rho'^2 / 2 = k^2 Omega(rho),
      Omega(rho) = rho (psi'(rho) - mu_M) - (p0(rho) - p_M)   (p0 = rho psi' - psi, Eq 10),
  zero at both Maxwell densities.  ``flat_profile`` integrates
  drho/dy = k sqrt(2 Omega / kappa_hat) outward from the mid density; the
  interface width (rho_l - rho_g) / max rho' is proportional to sqrt(kappa_hat)/k.
* ``derivative_errors`` applies each difference scheme (``lbm_gradient``, on the
  GPU) to the sampled profile of a periodic slab and reports the error against
  the analytic derivative, as in Fig 3(a).
* ``force_angles`` evaluates the nonideal force of the tanh droplet of Eq 26
  (``lbm_force``) and its angle deviation from the radial direction (Eq 30) and
  its error against the exact force of that field, as in Figs 5(b)-7.

* ``spurious_sweep`` runs the droplet of the benchmark (radius L/4, tanh width
  10, Tr = 0.7) with every scheme at a small and a large k for a fixed number
  of steps and reports the spurious current max|v| (Sec 3.3), the mass drift
  and the rate, or the step at which the run diverged.

Run ``python -m paper_2205_09186_amd.studies`` for the tables (JSON on stdout),
``python -m paper_2205_09186_amd.studies spurious --lattice D3Q19 --n 256`` for
the spurious-current sweep.
"""
from __future__ import annotations

import json
import math
import sys

import numpy as np

from . import lbm

CS2 = 1.0 / 3.0


class FlatInterface:
    """The equilibrium flat-interface profile of Eq 29 at (Tr, k, kappa_hat).

    The profile is built on the logistic coordinate u, rho = rho_g + (rho_l -
    rho_g) s(u), s = 1 / (1 + e^-u), which resolves both exponential tails:
    Omega(u) = int (psi'(rho) - mu_M) drho, from the gas end for u < 0 and from
    the liquid end for u > 0 (the two agree at u = 0 only at the Maxwell
    densities), then y(u) = int (drho/du) / rho'(rho) du from the mid point,
    both by cumulative Simpson sums on a fine grid."""

    def __init__(self, Tr: float, k: float, kappa: float, p: lbm.Params | None = None, U: float = 30.0,
                 h: float = 2e-3):
        from scipy.interpolate import CubicSpline
        self.Tr, self.k, self.kappa = Tr, k, kappa
        self.params = p or lbm.Params()
        self.rho_g, self.rho_l = lbm.coexistence(Tr, self.params)
        p0, mu = lbm.eos(np.array([self.rho_g, self.rho_l]), Tr, self.params)
        self.p_M, self.mu_M = float(p0[0]), float(mu[0])
        D = self.rho_l - self.rho_g
        m = int(round(U / h))
        u = np.linspace(-U, U, 2 * m + 1)
        sig = 0.5 * (1.0 + np.tanh(0.5 * u))
        rho = self.rho_g + D * sig
        drdu = D * sig * (1.0 - sig)
        _, mub = lbm.eos(rho, Tr, self.params)
        integrand = (mub - self.mu_M) * drdu
        # tails beyond |u| = U: Omega ~ psi''(rho_b) (rho - rho_b)^2 / 2, psi'' = p0'/rho
        def dmu(rb):
            e = 1e-6 * rb
            pp, _ = lbm.eos(np.array([rb + e, rb - e]), Tr, self.params)
            return (pp[0] - pp[1]) / (2 * e) / rb
        om = np.empty_like(u)
        gas = _cumsimpson(integrand[: m + 1], h) + 0.5 * dmu(self.rho_g) * (rho[0] - self.rho_g) ** 2
        liq = _cumsimpson(integrand[m:][::-1], -h)[::-1] + 0.5 * dmu(self.rho_l) * (rho[-1] - self.rho_l) ** 2
        om[: m + 1] = gas
        om[m:] = liq
        self.omega_mismatch = float(abs(gas[-1] - liq[0]) / max(abs(gas[-1]), 1e-300))
        slope = k * np.sqrt(2.0 * np.maximum(om, 0.0) / kappa)
        g = drdu / slope
        y = np.empty_like(u)
        y[m:] = _cumsimpson(g[m:], h)
        y[: m + 1] = -_cumsimpson(g[: m + 1][::-1], h)[::-1]
        self._u_of_y = CubicSpline(y, u)
        self._slope_of_u = CubicSpline(u, slope)
        self._D = D
        self._w = D / float(slope.max())
        # beyond the table the profile is the linearised tail:
        # rho - rho_b ~ exp(-|y| / lam_b), lam_b = sqrt(kappa_hat / psi''(rho_b)) / k
        self._ends = (float(y[0]), float(y[-1]), float(rho[0]), float(rho[-1]))
        self._lam = (math.sqrt(kappa / dmu(self.rho_g)) / k, math.sqrt(kappa / dmu(self.rho_l)) / k)

    def profile(self, d):
        """rho and rho' at signed distances d (liquid side positive) from the
        point where rho = (rho_g + rho_l) / 2."""
        d = np.asarray(d, dtype=np.float64)
        y0, y1, r0, r1 = self._ends
        u = self._u_of_y(np.clip(d, y0, y1))
        sig = 0.5 * (1.0 + np.tanh(0.5 * u))
        rho, slope = self.rho_g + self._D * sig, self._slope_of_u(u)
        lo, hi = d < y0, d > y1
        if lo.any():
            e = np.exp((d[lo] - y0) / self._lam[0]) * (r0 - self.rho_g)
            rho[lo], slope[lo] = self.rho_g + e, e / self._lam[0]
        if hi.any():
            e = np.exp(-(d[hi] - y1) / self._lam[1]) * (self.rho_l - r1)
            rho[hi], slope[hi] = self.rho_l - e, e / self._lam[1]
        return rho, slope

    def width(self):
        """(rho_l - rho_g) / max rho'."""
        return self._w


def _cumsimpson(f, h):
    """Cumulative integral of samples f (spacing h, signed) from the first
    sample, fourth order: each interval integrates the cubic through its four
    nearest samples, h/24 (-f[i-1] + 13 f[i] + 13 f[i+1] - f[i+2]), one-sided
    at the two ends."""
    n = f.size
    seg = np.empty(n - 1)
    if n < 4:
        seg[:] = 0.5 * h * (f[1:] + f[:-1])
    else:
        seg[1:-1] = h / 24.0 * (-f[:-3] + 13.0 * f[1:-2] + 13.0 * f[2:-1] - f[3:])
        seg[0] = h / 24.0 * (9.0 * f[0] + 19.0 * f[1] - 5.0 * f[2] + f[3])
        seg[-1] = h / 24.0 * (f[-4] - 5.0 * f[-3] + 19.0 * f[-2] + 9.0 * f[-1])
    out = np.zeros(n)
    out[1:] = np.cumsum(seg)
    return out


def slab_field(fi: FlatInterface, n: int):
    """A periodic slab of length n: liquid in the middle half, two interfaces.
    Returns rho[n] and the analytic d rho / dy[n]."""
    y = np.arange(n, dtype=np.float64)
    c = 0.5 * (n - 1)
    dist = 0.25 * n - np.abs(y - c)            # positive inside the liquid
    rho, slope = fi.profile(dist)
    return rho, slope * -np.sign(y - c)


def derivative_errors(Tr=0.6, ks=(0.1, 0.2, 0.3, 0.4, 0.6, 0.8, 1.0), kappa=0.04, n=256,
                      schemes=("CD2", "CD4", "CD6", "CFDS4", "CFDS6", "CFDS8", "OCFDS4")):
    """Max error of G[rho] against the analytic rho' over a periodic slab,
    relative to max |rho'| (Fig 3(a)), per scheme and k.  kappa_hat = 0.04
    puts the width between 25 nodes (k = 0.1) and 2.5 nodes (k = 1)."""
    import torch
    out = {}
    for k in ks:
        fi = FlatInterface(Tr, k, kappa)
        rho, drho = slab_field(fi, n)
        field = np.repeat(rho[:, None], 4, axis=1)             # (ny = n, nx = 4), uniform in x
        row = {}
        for s in schemes:
            p = lbm.Params(lattice=lbm.D2Q9, nx=4, ny=n, Tr=Tr, k=k, kappa=kappa, scheme=lbm.SCHEMES[s])
            sim = lbm.Simulation(p, field)
            g, _ = sim.gradient(torch.from_numpy(field.reshape(-1)))
            gy = g[1].cpu().numpy()[:, 0]
            row[s] = float(np.abs(gy - drho).max() / np.abs(drho).max())
            sim.close()
        out[f"{k:g}"] = {"width": fi.width(), "errors": row}
    return out


def exact_droplet_force(x, y, x0, y0, r0, W, rho_g, rho_l, Tr, k, kappa):
    """Exact nonideal force (Eq 12) of the 2D tanh droplet of Eq 26: every
    derivative of the radial profile in closed form, psi'' by Gibbs-Duhem
    (psi'' = p0'/rho) with p0' from a centred difference of the EOS."""
    r = np.hypot(x - x0, y - y0)
    A, B = 0.5 * (rho_l + rho_g), 0.5 * (rho_l - rho_g)
    s = 2.0 / W
    t = np.tanh(s * (r - r0))
    sech2 = 1.0 - t * t
    rho = A - B * t
    r1 = -B * s * sech2                                      # d rho / dr
    r2 = 2.0 * B * s * s * t * sech2                         # d2
    r3 = 2.0 * B * s ** 3 * sech2 * (sech2 - 2.0 * t * t)    # d3
    h = 1e-6 * rho
    p_hi, _ = lbm.eos(rho + h, Tr)
    p_lo, _ = lbm.eos(rho - h, Tr)
    dmu = (p_hi - p_lo) / (2.0 * h) / rho                    # psi''
    rr = np.maximum(r, 1.0)                                  # the centre node: no force (r1 ~ e^(-4 r0/W))
    dlap = r3 + r2 / rr - r1 / (rr * rr)                     # d/dr (rho'' + rho'/r)
    dmuhat = k * k * dmu * r1 - kappa * dlap
    Fr = np.where(r >= 1.0, -rho * dmuhat + CS2 * r1, 0.0)
    return Fr * (x - x0) / rr, Fr * (y - y0) / rr, rho


def force_angles(Tr=0.7, n=300, r0=60.0, W=10.0, k=0.16, kappa=0.004,
                 schemes=("CD2", "CD4", "CD6", "E4", "E6", "E8", "E10", "CFDS4", "CFDS6", "OCFDS4")):
    """Angle deviation (Eq 30) and relative error of the force of the Eq 26
    droplet, over nodes with |F| above 1% of its maximum."""
    g, l = lbm.coexistence(Tr)
    yy, xx = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
    x0 = y0 = n // 2
    Fx_e, Fy_e, rho = exact_droplet_force(xx, yy, x0, y0, r0, W, g, l, Tr, k, kappa)
    mag_e = np.hypot(Fx_e, Fy_e)
    sel = mag_e > 0.01 * mag_e.max()
    theta0 = np.arctan2(yy - y0, xx - x0)
    phi = np.degrees(theta0[sel]) % 90.0                     # position angle folded to [0, 90)
    out = {}
    for s in schemes:
        p = lbm.Params(lattice=lbm.D2Q9, nx=n, ny=n, Tr=Tr, k=k, kappa=kappa, scheme=lbm.SCHEMES[s])
        sim = lbm.Simulation(p, rho)
        F, _ = sim.force()
        sim.close()
        Fx, Fy = F[0][sel], F[1][sel]
        # the force points towards the centre: compare with the inward radial angle
        dth = np.angle(np.exp(1j * (np.arctan2(Fy, Fx) - np.arctan2(-(yy[sel] - y0), -(xx[sel] - x0)))))
        err = np.hypot(Fx - Fx_e[sel], Fy - Fy_e[sel]) / mag_e[sel].max()
        bins = {}
        for c in (0.0, 22.5, 45.0, 67.5):
            m = np.abs(((phi - c + 45.0) % 90.0) - 45.0) < 5.625
            bins[f"{c:g}"] = float(np.degrees(np.abs(dth[m])).mean())
        out[s] = {"max_dtheta_deg": float(np.degrees(np.abs(dth)).max()),
                  "rms_dtheta_deg": float(np.degrees(np.sqrt(np.mean(dth * dth)))),
                  "mean_abs_dtheta_deg_by_position_angle": bins,
                  "max_rel_force_error": float(err.max()), "rms_rel_force_error": float(np.sqrt(np.mean(err ** 2)))}
    return out


def spurious_sweep(lattice=lbm.D3Q19, n=256, steps=20000, ks=(0.1, 0.25), Tr=0.7, kappa=0.004,
                   schemes=("CD2", "CD4", "CD6", "E4", "E6", "E8", "OCFDS4", "CFDS4", "CFDS6", "CFDS8"),
                   check=1000):
    """The droplet of the benchmark (R = n/4, W = 10, seeded noise) with each
    scheme and k for `steps` steps: U = max|v| and mass every `check` steps;
    a non-finite state or U above the sound speed ends the run (diverged)."""
    import time
    import torch
    from . import inputs
    shape = (n, n, n) if lattice == lbm.D3Q19 else (n, n)
    g, l = lbm.coexistence(Tr)
    rho0 = inputs.droplet(shape, 0.25 * n, 10.0, g, l)
    out = []
    for k in ks:
        for sch in schemes:
            if sch == "E10" and lattice == lbm.D3Q19:
                continue
            p = lbm.Params(lattice=lattice, nx=n, ny=n, nz=(n if lattice == lbm.D3Q19 else 1), Tr=Tr, k=k,
                           kappa=kappa, scheme=lbm.SCHEMES[sch])
            sim = lbm.Simulation(p, torch.from_numpy(rho0.reshape(-1)).cuda())
            if sim.num_variants > 1:
                sim.tune(steps=3)
            U0, M0, _ = sim.spurious_max()
            done, U, M, status, hist = 0, U0, M0, "ran", []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            while done < steps:
                sim.step(min(check, steps - done))
                done += min(check, steps - done)
                U, M, _ = sim.spurious_max()
                hist.append(U)
                if not math.isfinite(U) or U > CS2 ** 0.5:
                    status = "diverged"
                    break
            wall = time.perf_counter() - t0
            row = dict(scheme=sch, k=k, kappa=kappa, Tr=Tr, steps=done, status=status, U=U,
                       mass_rel_drift=abs(M - M0) / M0, mlups=p.n * done / wall / 1e6, U_every_check=hist)
            print(json.dumps({key: row[key] for key in ("scheme", "k", "kappa", "Tr", "steps", "status", "U",
                                                        "mass_rel_drift", "mlups")}), file=sys.stderr, flush=True)
            out.append(row)
            sim.close()
            del sim
            torch.cuda.empty_cache()
    return out


def flat_interface_3d(Trs=(0.95, 0.9, 0.8, 0.7, 0.6, 0.5), schemes=("CD6", "OCFDS4"), H=400, w=10,
                      steps=150000, tau=0.8, k=0.1, kappa=0.004, check=10000):
    """The flat interface of Sec 3.4 in 3D: a D3Q19 w x w x H periodic box
    (the paper's 400 x 10 x 10), liquid in the middle half along the long axis
    (tanh edges of width 10, no noise), tau 0.8, k 0.1, run `steps` steps.
    Per run: status (a non-finite state or U above the sound speed ends it),
    U, and rho at the centre of the liquid and of the gas against the Maxwell
    densities."""
    import time
    from . import inputs
    rows = []
    for sname in schemes:
        for Tr in Trs:
            g, l = lbm.coexistence(Tr)
            rho0 = inputs.slab((H, w, w), 0, 10.0, g, l, amplitude=0.0)
            p = lbm.Params(lattice=lbm.D3Q19, nx=w, ny=w, nz=H, tau=tau, Tr=Tr, k=k, kappa=kappa,
                           scheme=lbm.SCHEMES[sname])
            sim = lbm.Simulation(p, rho0)
            done, status, U = 0, "ran", 0.0
            t0 = time.perf_counter()
            while done < steps:
                n = min(check, steps - done)
                sim.step(n)
                done += n
                U, _, code = sim.spurious_max()
                if code != 0 or not math.isfinite(U):
                    status = "diverged"
                    break
            wall = time.perf_counter() - t0
            row = dict(scheme=sname, Tr=Tr, status=status, steps=done, U=U, rho_l_maxwell=l, rho_g_maxwell=g,
                       mlups=p.n * done / wall / 1e6)
            if status == "ran":
                r = sim.macros()[0]
                row.update(rho_l=float(r[H // 2, w // 2, w // 2]), rho_g=float(r[0, w // 2, w // 2]))
                row.update(rel_l=row["rho_l"] / l - 1.0, rel_g=row["rho_g"] / g - 1.0)
            print(json.dumps({key: row[key] for key in row}), file=sys.stderr, flush=True)
            rows.append(row)
            sim.close()
    return rows


def low_temperature_envelope(Trs=(0.3, 0.4, 0.5), widths=(5.0, 10.0, 20.0, 35.0), steps=20000,
                             schemes=("CD4", "CD6", "OCFDS4")):
    """Which interface widths keep low-temperature runs finite: 2D droplets
    (256^2, R 64) and slabs (8 x 512) whose Eq 29 width W is set either
    through kappa_hat at k = 0.1 or through k at kappa_hat = 0.004 and 0.001
    (W = sqrt(kappa_hat) W1 / k, W1 the width at k = kappa_hat = 1), tanh
    starts of width W, SRT, all run together on the batched kernel.  Per
    instance: status, U, and the centre / edge densities against Maxwell."""
    from . import inputs
    rows, ps, rs = [], [], []
    for Tr in Trs:
        w1 = FlatInterface(Tr, 1.0, 1.0).width()
        g, l = lbm.coexistence(Tr)
        combos = [(W, (W * 0.1 / w1) ** 2, 0.1, "kappa") for W in widths]
        combos += [(W, kap, math.sqrt(kap) * w1 / W, "k") for kap in (0.004, 0.001) for W in widths]
        for W, kap, k, via in combos:
            for sname in schemes:
                for kind in ("drop", "slab"):
                    shape = (256, 256) if kind == "drop" else (512, 8)
                    if kind == "drop":
                        r = inputs.droplet(shape, 64.0, W, g, l, instance_id=len(rows), relative=True)
                    else:
                        r = inputs.slab(shape, 0, W, g, l, instance_id=len(rows), relative=True)
                    ps.append(lbm.Params(lattice=lbm.D2Q9, nx=shape[1], ny=shape[0], Tr=Tr, k=k, kappa=kap,
                                         scheme=lbm.SCHEMES[sname]))
                    rs.append(r)
                    rows.append(dict(kind=kind, Tr=Tr, W=W, via=via, kappa=kap, k=k, scheme=sname,
                                     rho_g_maxwell=g, rho_l_maxwell=l))
    b = lbm.Batch(ps, rs)
    b.set_form(lbm.BATCH_PHASES)
    st, done, U = b.run(steps, check_every=100, tol=0.0, chunk=min(steps, 2000))
    for i, row in enumerate(rows):
        row.update(status=["running", "converged", "diverged"][int(st[i])], steps=int(done[i]), U=float(U[i]))
        if st[i] != lbm.DIVERGED:
            r = b.instance(i).macros()[0]
            c = (128, 128) if row["kind"] == "drop" else (256, 0)
            row.update(rho_l=float(r[c]), rho_g=float(r[0, 0]))
    b.close()
    return rows


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "slab3d":
        json.dump(flat_interface_3d(), sys.stdout)
        print()
        return
    if len(sys.argv) > 1 and sys.argv[1] == "lowt":
        json.dump(low_temperature_envelope(), sys.stdout)
        print()
        return
    if len(sys.argv) > 1 and sys.argv[1] == "spurious":
        import argparse
        ap = argparse.ArgumentParser()
        ap.add_argument("cmd")
        ap.add_argument("--lattice", default="D3Q19", choices=["D2Q9", "D3Q19"])
        ap.add_argument("--n", type=int, default=256)
        ap.add_argument("--steps", type=int, default=20000)
        ap.add_argument("--schemes", default="")
        ap.add_argument("--ks", default="0.1,0.25")
        ap.add_argument("--Tr", type=float, default=0.7)
        ap.add_argument("--kappa", type=float, default=0.004)
        ap.add_argument("--check", type=int, default=1000)
        a = ap.parse_args()
        lat = lbm.D3Q19 if a.lattice == "D3Q19" else lbm.D2Q9
        kw = dict(lattice=lat, n=a.n, steps=a.steps, ks=tuple(float(x) for x in a.ks.split(",")), Tr=a.Tr,
                  kappa=a.kappa, check=a.check)
        if a.schemes:
            kw["schemes"] = tuple(a.schemes.split(","))
        json.dump(spurious_sweep(**kw), sys.stdout)
        print()
        return
    res = {"derivative_errors_Tr0.6": derivative_errors(), "force_angles_Tr0.7": force_angles()}
    widths = {f"{k:g}": FlatInterface(0.6, k, 0.04).width() for k in (0.1, 0.2, 0.4, 0.8, 1.0)}
    res["width_vs_k_Tr0.6"] = widths
    json.dump(res, sys.stdout, indent=1)
    print()


if __name__ == "__main__":
    main()
