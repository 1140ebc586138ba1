"""What the trained network gains over the method without it: held-out D2Q9
droplets started from the tanh profile of Eq 26 (width 10) and from the
shipped network's profile (learned_net.npy, mass-matched by the radius), both
run by the batched kernel until |U(t) - U(t - 100)| < 1e-12 (U = max |v|,
checked every 100 steps).  The droplets are drawn with a seed disjoint from
the training and earlier evaluation sets, each scheme in the temperature range
where it runs under SRT."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NET = os.path.join(ROOT, "paper_2205_09186_amd", "learned_net.npy")


def test_learned_start_against_tanh_start():
    import torch
    from paper_2205_09186_amd import lbm, learned
    net = learned.Net(0)
    net.load(np.load(NET))
    specs = learned.droplet_set(16, seed=60, lmax=128)
    ps, rs = learned._tanh_batch(specs)
    starts, fallback = [], 0
    for p, r, d in zip(ps, rs, specs):
        g, l = lbm.coexistence(d["Tr"])
        rho, _ = learned.mass_matched_field(net, p, d["R"], d["Tr"], d["k"], d["scheme"], g, l, float(r.sum()))
        if rho is None or not bool(torch.isfinite(rho).all()):
            fallback += 1
            starts.append(r)
        else:
            starts.append(rho.cpu().numpy().reshape(r.shape))
    res = {}
    for name, rhos in (("tanh", rs), ("learned", starts)):
        print(f"case learned-start gain: {name} start, 16 droplets", flush=True)
        b = lbm.Batch(ps, rhos)
        st, steps, U = b.run(300000, check_every=100, tol=1e-12, chunk=20000)
        dens = []
        for i, d in enumerate(specs):
            rr = b.instance(i).macros()[0]
            dens.append((float(rr[d["L"] // 2, d["L"] // 2]), float(rr[0, 0])))
        res[name] = (st, steps, U, dens)
        b.close()
    t, lrn = res["tanh"], res["learned"]
    rows = []
    for i, d in enumerate(specs):
        ok = t[0][i] == lbm.CONVERGED and lrn[0][i] == lbm.CONVERGED
        drop = ok and t[3][i][0] > 1.5 * t[3][i][1] and lrn[3][i][0] > 1.5 * lrn[3][i][1]
        line = (f"  droplet {i}: L={d['L']} R={d['R']:.1f} scheme={learned.SCHEMES6.index(d['scheme'])} "
                f"Tr={d['Tr']:.3f} k={d['k']:.3f} status {t[0][i]}/{lrn[0][i]} steps {t[1][i]}/{lrn[1][i]}")
        if drop:
            rows.append(dict(ratio=lrn[1][i] / t[1][i], dU=abs(lrn[2][i] - t[2][i]) / abs(t[2][i]),
                             dl=abs(lrn[3][i][0] - t[3][i][0]) / t[3][i][0],
                             dg=abs(lrn[3][i][1] - t[3][i][1]) / t[3][i][1]))
            line += f" ratio {rows[-1]['ratio']:.3f} dU {rows[-1]['dU']:.1e}"
        print(line, flush=True)
    ratio = np.array([r["ratio"] for r in rows])
    dU = np.array([r["dU"] for r in rows])
    print(f"case learned-start gain: fallback {fallback}, compared {len(rows)}, median steps ratio "
          f"{np.median(ratio):.4f}, learned faster in {(ratio < 1).sum()}, total steps saved "
          f"{1 - sum(lrn[1][i] for i in range(16)) / sum(t[1][i] for i in range(16)):.4f}; final U rel diff median "
          f"{np.median(dU):.2e} max {dU.max():.2e}, within 1e-6: {(dU <= 1e-6).sum()}; rho_l rel diff max "
          f"{max(r['dl'] for r in rows):.2e}, rho_g rel diff max {max(r['dg'] for r in rows):.2e}", flush=True)
    # near the critical point some droplets dissolve into the vapour of their
    # box from either start; those end in different states and are not compared
    assert fallback <= 4
    assert len(rows) >= 8
    assert np.median(ratio) < 1.0
    assert max(r["dl"] for r in rows) < 1e-6
    assert max(r["dg"] for r in rows) < 1e-5
    assert np.median(dU) < 1e-6
