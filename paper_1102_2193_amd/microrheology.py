"""Active microrheology of a colloid in a nematic (Sec. 3.1, Fig. 3).

A colloid with planar (tangential) anchoring sits in a nematic whose far
field lies along z.  After the director field has settled around the fixed
colloid, the colloid is released (free motion) and pulled with a constant
force f along (z) or perpendicular to (x) the far-field director; the
paper finds that it moves faster along the director, the ratio of the two
effective viscosities being about 1.85.

The box is periodic, so a constant pull alone would make the total
momentum grow without bound: the fluid nodes carry a uniform opposite
force, -f / (number of fluid nodes), so that the total is zero and the
colloid reaches a steady speed relative to a fluid at rest on average.
The settled state is carried from the context without that force to the
one with it through lc_get_state / lc_set_state.

Material parameters are the paper's (A0 = 1, gamma = 3, K = 0.065,
xi = 0.7, Gamma = 0.5) with eta = 0.1 (tau = 0.8); the box size, settling
time and run length are choices of this reproduction (the paper does not
give them).
"""
import argparse
import json
import math
import sys

import numpy as np

from . import inputs

PARAMS = dict(inputs.PAPER_CHOLESTERIC, tau=0.8)
Q_EQ = 0.5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pull(L=128, a=16.0, f=0.09, settle=2000, steps=16000, every=500, tile=None):
    """Speed of the pulled colloid along and perpendicular to the director:
    {"along": [(step, v)], "perp": [...]}, with the settled state shared."""
    from . import lc
    centre = (0.5 * L,) * 3
    base = dict(nx=L, precision="fp32", **PARAMS)
    ctx = lc.Context([base])
    if tile is not None:
        ctx.set_tile(tile)
    ctx.set_colloid(0, centre, a, anchoring="planar", W=math.inf, S0=Q_EQ)
    ctx.set_Q(0, inputs.uniaxial_q(L, L, L, Q_EQ, director=(0.0, 0.0, 1.0)))
    log("settling %d steps (fixed colloid)" % settle)
    ctx.step(settle)
    state = ctx.get_state()
    nf = int((ctx.solid_id(0) == 0).sum())   # fluid nodes, from the library's solid map
    ctx.close()
    out = {}
    for name, axis in (("along", 2), ("perp", 0)):
        fext = [0.0, 0.0, 0.0]
        fext[axis] = f
        body = [0.0, 0.0, 0.0]
        body[axis] = -f / nf
        c2 = lc.Context([dict(base, body_force=tuple(body))])
        if tile is not None:
            c2.set_tile(tile)
        c2.set_state(state)
        c2.set_colloid(0, centre, a, anchoring="planar", W=math.inf, S0=Q_EQ, motion=lc.FREE,
                       fext=tuple(fext), rho_c=PARAMS["rho0"])
        series = []
        for k in range(steps // every):
            c2.step(every)
            series.append(((k + 1) * every, float(c2.get_colloid(0).vel[axis])))
        log("%s: v(%d) = %.4e" % (name, steps, series[-1][1]))
        out[name] = series
        c2.close()
    return out


def summary(res, f, a, eta=(PARAMS["tau"] - 0.5) / 3.0):
    """Steady speeds (mean over the last quarter of the samples), their ratio,
    the drag coefficients of the linear drag law f = A v that the paper fits
    (A along and across the director; it prints 63.2 and 116.9) and the
    effective viscosities of Stokes' law f = 6 pi eta_eff a v (no correction
    for the periodic images)."""
    def steady(series):
        v = np.array([s[1] for s in series])
        return float(np.mean(v[-max(1, len(v) // 4):]))
    va, vp = steady(res["along"]), steady(res["perp"])
    return {"v_along": va, "v_perp": vp, "ratio_along_over_perp": va / vp,
            "drag_along": f / va, "drag_perp": f / vp,
            "eta_eff_along": f / (6 * math.pi * a * va), "eta_eff_perp": f / (6 * math.pi * a * vp),
            "eta": eta, "paper_ratio": 1.85, "paper_drag_along": 63.2, "paper_drag_perp": 116.9}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--a", type=float, default=16.0)
    ap.add_argument("--f", type=float, default=0.09)
    ap.add_argument("--settle", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=16000)
    ap.add_argument("--every", type=int, default=500)
    args = ap.parse_args(argv)
    res = pull(args.L, args.a, args.f, args.settle, args.steps, args.every)
    out = {"args": vars(args), "series": res, "summary": summary(res, args.f, args.a)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
