"""What the trained warm start gains over the plain helix start (GPU).

Two held-out cases (not in the training seeds): seed 9010 (planar, pitch
25.6, a = 7.37) and seed 9042 (normal, pitch 16, a = 8.88), 64^3, the
paper's cholesteric parameters, flow off.  The plain relaxation from the
helix, run until converged, defines F*; started from the network's
prediction the same relaxation must reach |F - F*| <= 1e-4 |F*| in fewer
steps and end in the same minimum (no fallback).
"""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_warm_start_reaches_the_relaxed_free_energy_sooner():
    from paper_1102_2193_amd import inputs, nn
    from paper_1102_2193_amd import warmstart as ws
    print("case: warm start vs plain, seeds 9010 and 9042, 64^3", flush=True)
    sys.stdout.flush()
    net = nn.Net(64)
    ws.load_weights(net, ws.WEIGHTS)
    cases = [inputs.warmstart_case(s) for s in (9010, 9042)]
    held = ws.relaxed_states(cases, 64, 60000, 2, 0, None, "plain")
    assert all(d["conv"] is not None for d in held)
    rows = ws.compare(net, held, 64, 60000, 0, None, 2)
    for r in rows:
        print("   seed %d: plain %d steps, warm %s steps, Q error helix %.2e warm %.2e" % (
            r["seed"], r["n_plain"], r["n_warm"], r["q_err_helix"], r["q_err_warm"]), flush=True)
        assert not r["fallback"]
        assert r["n_warm"] < r["n_plain"]
        assert r["q_err_warm"] < 0.5 * r["q_err_helix"]
    assert ws.summary(rows)["ratio_of_means"] < 0.25


def test_fluid_masks_count_lattice_points_outside_the_sphere():
    """The warm start's loss mask comes from the library's solid map; it
    counts the lattice points with |x - R|^2 >= a^2 (brute force)."""
    import numpy as np
    from paper_1102_2193_amd import warmstart as ws
    print("case: fluid masks of three radii on 32^3", flush=True)
    masks = ws.fluid_masks([{"a": a} for a in (3.0, 4.5, 7.3)], 32)
    r = np.arange(-16, 16)
    for a, m in zip((3.0, 4.5, 7.3), masks):
        inside = sum(1 for x in r for y in r for z in r if x * x + y * y + z * z < a * a)
        assert m.size - int(m.sum()) == inside
