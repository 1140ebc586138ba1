"""Uneven droplet / flat-slab sweep over reduced temperature, radius, scheme and
k, run by the batched persistent kernel (the runs behind the coexistence curve
of Sec 3.4 and the spurious-current comparisons of Sec 3.3).

Instances: 48 flat slabs 8 x H (H uniform over multiples of 8 in [128, 1024])
and 48 droplets of radius R in [10, 60] on L x L (L uniform over multiples of 8
in [max(64, 2R + 64), 256]); Tr uniform in [0.2, 0.95]; k uniform in [0.1,
0.25]; scheme uniform over CD2, CD4, CD6, E4, E8, OCFDS4; tanh width 10;
relative noise +-1e-6 (absolute noise would make the gas density negative
below Tr ~ 0.45).  Each
instance runs until |U(t) - U(t - 100)| < 1e-10 (checked every 100 steps),
until it diverges, or until the step cap.  --collision mrt runs every
instance with the MRT collision of Eq 3-5 (the paper's own runs) instead of
BGK.  The tuner picks the launch form; --time-forms times both.

``python -m paper_2205_09186_amd.sweep`` prints one JSON summary.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs, lbm

SCHEMES6 = [lbm.CD2, lbm.CD4, lbm.CD6, lbm.E4, lbm.E8, lbm.OCFDS4]
NAMES = {v: k for k, v in lbm.SCHEMES.items()}


def build(n_slabs=48, n_drops=48, seed=0, kappa=0.004, width=10.0, tr_range=(0.2, 0.95), k_range=(0.1, 0.25),
          collision=0):
    descs = inputs.sweep_instances(n_slabs, n_drops, seed=seed, n_schemes=6, tr_range=tr_range, k_range=k_range)
    params, rhos = [], []
    for d in descs:
        d["scheme"] = SCHEMES6[d["scheme"]]
        g, l = lbm.coexistence(d["Tr"])
        d["rho_g_maxwell"], d["rho_l_maxwell"] = g, l
        if d["kind"] == "slab":
            r = inputs.slab((d["ny"], d["nx"]), 0, width, g, l, instance_id=d["instance_id"], relative=True)
        else:
            r = inputs.droplet((d["ny"], d["nx"]), d["radius"], width, g, l, instance_id=d["instance_id"],
                               relative=True)
        params.append(lbm.Params(lattice=lbm.D2Q9, nx=d["nx"], ny=d["ny"], Tr=d["Tr"], k=d["k"], kappa=kappa,
                                 scheme=d["scheme"], collision=collision))
        rhos.append(r)
    return descs, params, rhos


def coexistence_of(view, d):
    """(rho_l, rho_g) of an instance: centre and edge of a slab; centre node and
    the node farthest from the centre of a droplet."""
    r = view.macros()[0]
    if d["kind"] == "slab":
        return float(r[d["ny"] // 2, 0]), float(r[0, 0])
    return float(r[d["ny"] // 2, d["nx"] // 2]), float(r[0, 0])


def run(max_steps=150000, check_every=100, tol=1e-10, chunk=2000, tune=True, form=None, **kw):
    """form: None lets the tuner choose (with tune=True), else
    lbm.BATCH_PERSISTENT or lbm.BATCH_PHASES."""
    descs, params, rhos = build(**kw)
    b = lbm.Batch(params, rhos)
    tuned = b.tune(steps=20, forms=(form,) if form is not None else (lbm.BATCH_PERSISTENT, lbm.BATCH_PHASES)) \
        if tune else None
    if form is not None:
        b.set_form(form)
    t0 = time.perf_counter()
    st, steps, U = b.run(max_steps, check_every=check_every, tol=tol, chunk=chunk)
    wall = time.perf_counter() - t0
    out = []
    for i, d in enumerate(descs):
        rec = dict(kind=d["kind"], nx=d["nx"], ny=d["ny"], Tr=round(d["Tr"], 4), k=round(d["k"], 4),
                   scheme=NAMES[d["scheme"]], radius=round(d["radius"], 2),
                   status=["running", "converged", "diverged"][int(st[i])], steps=int(steps[i]), U=float(U[i]))
        if st[i] != lbm.DIVERGED:
            rl, rg = coexistence_of(b.instance(i), d)
            rec.update(rho_l=rl, rho_g=rg, rho_l_maxwell=d["rho_l_maxwell"], rho_g_maxwell=d["rho_g_maxwell"])
        out.append(rec)
    # node updates actually performed (tuning steps excluded)
    nodes = np.array([p.n for p in params], dtype=np.float64)
    return {"instances": out, "wall_s": wall, "node_updates": float((nodes * np.array(steps)).sum()),
            "form": ["persistent", "phases"][b.form], "block": b.block, "launch": b.launch_mode,
            "tuner_ms_per_step": tuned, "counts": {s: sum(1 for r in out if r["status"] == s)
                                                   for s in ("running", "converged", "diverged")}}


def time_forms(steps=1000, warm=200, check_every=100, block=512, **kw):
    """ms per step of each launch form on the same set with every instance
    running (tol 0, one chunk of `steps` after `warm` untimed steps that also
    capture the launch graph)."""
    import torch
    descs, params, rhos = build(**kw)
    out = {}
    for form, name in ((lbm.BATCH_PERSISTENT, "persistent"), (lbm.BATCH_PHASES, "phases")):
        b = lbm.Batch(params, rhos)
        b.set_block(block)
        b.set_form(form)
        b.run(warm, check_every=check_every, tol=0.0, chunk=warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(steps, check_every=check_every, tol=0.0, chunk=steps)
        ms = (time.perf_counter() - t0) * 1e3 / steps
        nodes = sum(p.n for p in params)
        out[name] = {"ms_per_step": round(ms, 4), "mlups": round(nodes / ms / 1e3, 1), "launch": b.launch_mode}
        b.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-steps", type=int, default=150000)
    ap.add_argument("--chunk", type=int, default=2000)
    ap.add_argument("--slabs", type=int, default=48)
    ap.add_argument("--drops", type=int, default=48)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--collision", default="srt", choices=["srt", "mrt"],
                    help="BGK (Eq 1 with one rate) or the D2Q9 MRT of Eq 3-5")
    ap.add_argument("--form", default="tune", choices=["tune", "persistent", "phases"],
                    help="batch launch form (default: the tuner's choice)")
    ap.add_argument("--time-forms", action="store_true",
                    help="only time the two launch forms (1000 steps each, every instance running)")
    a = ap.parse_args()
    if a.time_forms:
        print(json.dumps(time_forms(n_slabs=a.slabs, n_drops=a.drops, seed=a.seed)))
        return
    form = {"tune": None, "persistent": lbm.BATCH_PERSISTENT, "phases": lbm.BATCH_PHASES}[a.form]
    res = run(max_steps=a.max_steps, chunk=a.chunk, n_slabs=a.slabs, n_drops=a.drops, seed=a.seed,
              collision=1 if a.collision == "mrt" else 0, form=form)
    res["collision"] = a.collision
    res["mlups"] = res["node_updates"] / res["wall_s"] / 1e6
    print(json.dumps(res))


if __name__ == "__main__":
    main()
