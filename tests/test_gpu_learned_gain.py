"""What the trained network gains over the method without it: held-out D2Q9
droplets started from the tanh profile of Eq 26 (width 10) and from the
shipped network's profile (learned_net.npy, mass-matched by the radius), both
run by the batched kernel until |U(t) - U(t - 100)| < 1e-14 (U = max |v|,
checked every 100 steps; at most 400,000 steps).  A criterion this tight lets
both starts settle on the same state, so the final spurious current is held to
the 1e-6 relative agreement asked of the learned start for every droplet
compared (at 1e-12 one slowly drifting E4 droplet still differed by 3e-4).
The droplets are drawn with a seed disjoint from the training and earlier
evaluation sets, each scheme in the temperature range where it runs under SRT
(learned.gain)."""
import pytest

pytestmark = pytest.mark.gpu


def test_learned_start_against_tanh_start():
    from paper_2205_09186_amd import learned
    print("case learned-start gain: 16 droplets, tanh and learned starts", flush=True)
    sm, rows = learned.gain(n=16, seed=60, lmax=128, tol=1e-14, max_steps=400000)
    for i, r in enumerate(rows):
        line = (f"  droplet {i}: L={r['L']} R={r['R']:.1f} scheme={r['scheme']} Tr={r['Tr']:.3f} k={r['k']:.3f} "
                f"status {r['status'][0]}/{r['status'][1]} steps {r['steps'][0]}/{r['steps'][1]}")
        if "ratio" in r:
            line += f" ratio {r['ratio']:.3f} dU {r['dU']:.1e}"
        print(line, flush=True)
    print(f"case learned-start gain: {sm}", flush=True)
    # near the critical point some droplets dissolve into the vapour of their
    # box from either start; those end in different states and are not compared
    assert sm["fallback"] <= 4
    assert sm["compared"] >= 8
    assert sm["steps_ratio_median"] < 1.0
    assert sm["rho_l_reldiff_max"] < 1e-6
    assert sm["rho_g_reldiff_max"] < 1e-6
    assert sm["U_reldiff_max"] <= 1e-6
