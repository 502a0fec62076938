"""Learned warm start of cholesteric relaxations around a fixed colloid.

The plain method relaxes a cholesteric around a colloid with normal or
planar anchoring from the uniform helix along z (Sec. 3 of Lintuvuori et
al.; material parameters of that section: A0 = 1, K = 0.065, gamma = 3,
chirality 0.3 at pitch 32).  A small 3D network (include/lc_nn.h) predicts
the relaxed Q field from radius, pitch and anchoring; its prediction is the
initial Q of the same relaxation, which stays the judge of the result.

Every lattice step and every network pass runs in the library's HIP
kernels; this module only orchestrates them:

* ``relax``: batched relaxations (one context, one L^3 box per case, colloid
  fixed at the box centre, W = infinity) with the library's step, by default
  with the flow switched off (pure Beris-Edwards relaxation: the free-energy
  minima do not depend on the flow, and with the flow on, helices of pitch
  21 and below leave the helix branch through instabilities that rounding
  seeds, so their end state is not a function of the inputs);
  F_d of every box sampled every ``every`` steps.
* ``train``: the network fitted to relaxed Q fields on the GPU, one case per
  Adam step (loss: mean over fluid sites of |Q_warm - Q*|_F^2).
* ``evaluate``: held-out cases relaxed from the helix until converged define
  F*; the same cases started from the prediction run as many steps.

Definitions used throughout:

* converged at step n: |F(m) - F(m - 1000)| < 1e-7 |F(m)| at every sample
  m in [n - 4000, n] (held for 4000 steps, so that a turning point of a slow
  oscillation does not count);
* steps-to-relax: the first sampled n after which |F - F*| <= 1e-4 |F*|
  holds at every later sample up to the plain run's convergence step;
* fallback: a warm run outside that band at the plain run's convergence step
  (a different minimum, not yet relaxed, or non-finite) is replaced by the
  plain run and charged its own steps plus the plain run's.

Command line:
  python -m paper_1102_2193_amd.warmstart train --out DIR [--ntrain N ...]
  python -m paper_1102_2193_amd.warmstart evaluate --weights W --out DIR
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import inputs, lc, nn

PARAMS = inputs.PAPER_CHOLESTERIC
Q_EQ = 0.5            # bulk order at gamma = 3
CONV_TOL = 1e-7
CONV_WINDOW = 1000
CONV_HOLD = 4000
BAND = 1e-4
EVERY = 100
TRAIN_SEED0 = 5000
HELD_SEED0 = 9000
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_net.lcnn")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def nn_case(c, L):
    return nn.make_case((0.5 * L,) * 3, c["a"], c["pitch"], c["anchoring"], inputs.Q_INIT, Q_EQ)


def helix(c, L):
    return inputs.helix_q(L, L, L, 2 * math.pi / c["pitch"], inputs.Q_INIT)


def fluid_masks(cases, L, chunk=32):
    """Fluid sites (1) of each case's colloid (radius c["a"], centred at
    (L/2)^3), from the library's own solid map (lc_get_solid)."""
    out = []
    for i in range(0, len(cases), chunk):
        part = cases[i:i + chunk]
        ctx = lc.Context([dict(nx=L, precision="fp32", hydro=0, **PARAMS) for _ in part])
        for b, c in enumerate(part):
            ctx.set_colloid(b, (0.5 * L,) * 3, c["a"], anchoring="normal", W=math.inf, S0=Q_EQ)
        out.extend((ctx.solid_id(b) == 0).astype(np.uint8) for b in range(len(part)))
        ctx.close()
    return out


def fluid_mask(c, L):
    return fluid_masks([c], L)[0]


def make_context(cases, L=64, hydro=0, tile=None):
    boxes = [dict(nx=L, precision="fp32", hydro=hydro, **dict(PARAMS, q0=2 * math.pi / c["pitch"]))
             for c in cases]
    ctx = lc.Context(boxes)
    if tile is not None:
        ctx.set_tile(tile)
    for b, c in enumerate(cases):
        ctx.set_colloid(b, (0.5 * L,) * 3, c["a"], anchoring=c["anchoring"], W=math.inf, S0=Q_EQ)
    return ctx


def pick_tile(n, L=64, hydro=0):
    """Fastest tile shape for n boxes of L^3, timed on a scratch context."""
    from . import tune
    cases = [{"a": 6.0, "pitch": 32.0, "anchoring": "normal"}] * n
    ctx = make_context(cases, L, hydro)
    for b in range(n):
        ctx.set_Q(b, helix(cases[b], L))
    res = tune.tune(ctx, steps=20, warm=4)
    ctx.close()
    return min(res, key=res.get), res


class Track:
    """F samples of one run (one every EVERY steps, the first at step 0) and
    its convergence step (definitions above)."""

    def __init__(self, F0):
        self.F = [F0]
        self.held = 0
        self.conv = None
        self.n = 0

    def add(self, f):
        self.n += EVERY
        self.F.append(f)
        k, lag = len(self.F) - 1, CONV_WINDOW // EVERY
        if k >= lag and abs(self.F[k] - self.F[k - lag]) < CONV_TOL * abs(self.F[k]):
            self.held += 1
        else:
            self.held = 0
        if self.conv is None and (self.held - 1) * EVERY >= CONV_HOLD:
            self.conv = self.n


def relax(cases, L=64, cap=60000, hydro=0, net=None, horizon=None, tile=None, label="relax"):
    """Run the boxes of ``cases`` together from the helix (net None) or
    from the network's prediction.  Stops when every box has converged (or,
    if ``horizon`` is given, when the run has reached max(horizon)), or at
    ``cap`` steps.  Returns the context, F samples [box][k] at steps
    k * EVERY, the convergence step of every box (None if not converged) and
    whether every step succeeded."""
    ctx = make_context(cases, L, hydro, tile)
    for b, c in enumerate(cases):
        if net is None:
            ctx.set_Q(b, helix(c, L))
        else:
            net.warm_start(nn_case(c, L), ctx, b)
    nb = len(cases)
    tr = [Track(ctx.diag(b)["free_energy"]) for b in range(nb)]
    n, t0, last = 0, time.time(), time.time()
    ok = True
    end = cap if horizon is None else min(cap, max(horizon))
    while n < end:
        try:
            ctx.step(EVERY)
        except lc.LCError as e:
            log("  %s: step %d failed (%s)" % (label, n + EVERY, e))
            ok = False
            break
        n += EVERY
        for b in range(nb):
            tr[b].add(ctx.diag(b)["free_energy"])
        done = n >= end or (horizon is None and all(t.conv is not None for t in tr))
        if time.time() - last > 30 or done:
            last = time.time()
            log("  %s: step %d, %d/%d converged, %.0f s" % (label, n, sum(t.conv is not None for t in tr), nb,
                                                              time.time() - t0))
        if done:
            break
    return ctx, [np.array(t.F) for t in tr], [t.conv for t in tr], ok


def box_counts(pitches, nbox):
    """Boxes per pitch for a pool of nbox boxes: proportional to the number
    of cases of each pitch (largest remainders), at least one and at most
    that number.  pitches: the case pitches (one entry per case)."""
    kinds = sorted(set(pitches))
    count = {p: pitches.count(p) for p in kinds}
    nbox = max(len(kinds), min(nbox, len(pitches)))
    share = {p: nbox * count[p] / len(pitches) for p in kinds}
    out = {p: max(1, min(count[p], int(share[p]))) for p in kinds}
    for p in sorted(kinds, key=lambda p: share[p] - int(share[p]), reverse=True):
        if sum(out.values()) >= nbox:
            break
        if out[p] < count[p]:
            out[p] += 1
    return out


def stream(cases, L, cap, nbox, hydro, tile, label, net=None, horizons=None, keep_Q=True):
    """Relax every case on a pool of boxes of one context, each box taking
    the next case of its pitch (the material of a box is fixed) as soon as
    its run ends: converged, at the case's horizon (if given) or at the cap.
    A box gives the same bits alone or in a batch and a new case starts from
    a fresh state (helix or prediction; fluid at rest), so each result is the
    one a batched run gives.  If a step fails (non-finite values flag the
    whole context), the running cases are marked failed and the pool goes on
    in a new context; plain runs (net None) raise instead.  Returns one dict
    per case, in input order: F samples, convergence step, ok, and the
    final Q with keep_Q."""
    pitches = [c["pitch"] for c in cases]
    counts = box_counts(pitches, nbox)
    queue = {p: [i for i, c in enumerate(cases) if c["pitch"] == p] for p in counts}
    box_pitch = [p for p in sorted(counts) for _ in range(counts[p])]
    nb = len(box_pitch)
    results = [None] * len(cases)
    t0, last = time.time(), time.time()

    def new_context():
        firsts = [cases[queue[p][0]] if queue[p] else {"pitch": p, "a": 4.0, "anchoring": "normal"} for p in box_pitch]
        return make_context(firsts, L, hydro, tile)

    ctx = new_context()
    run = [None] * nb      # (case index, Track, end step)
    rest = None

    def start(b):
        p = box_pitch[b]
        if not queue[p]:
            run[b] = None
            return
        i = queue[p].pop(0)
        c = cases[i]
        ctx.set_colloid(b, (0.5 * L,) * 3, c["a"], anchoring=c["anchoring"], W=math.inf, S0=Q_EQ)
        if net is None:
            ctx.set_Q(b, helix(c, L))
        else:
            net.warm_start(nn_case(c, L), ctx, b)
        if hydro:
            nonlocal rest
            if rest is None:
                # fluid at rest, f = w_i rho0 (D3Q19 weights in the order of lc.h)
                w = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)
                rest = np.broadcast_to(w.reshape(19, 1, 1, 1) * PARAMS.get("rho0", 1.0), (19, L, L, L)).copy()
            ctx.set_f(b, rest)
            ctx.set_u(b, np.zeros((3, L, L, L)))
        end = cap if horizons is None else min(cap, horizons[i])
        run[b] = (i, Track(ctx.diag(b)["free_energy"]), end)

    def finish(b, ok):
        i, tr, _ = run[b]
        res = {"F": np.array(tr.F), "conv": tr.conv, "ok": ok}
        if keep_Q and ok:
            res["Q"] = ctx.get_Q(b)
        results[i] = res

    for b in range(nb):
        start(b)
    while any(r is not None for r in run):
        try:
            ctx.step(EVERY)
        except lc.LCError as e:
            if net is None:
                raise RuntimeError("%s: a plain relaxation failed (%s)" % (label, e))
            log("  %s: step failed (%s); %d running cases marked failed" % (label, e, sum(r is not None for r in run)))
            for b in range(nb):
                if run[b] is not None:
                    finish(b, False)
            ctx.close()
            ctx = new_context()
            for b in range(nb):
                start(b)
            continue
        for b in range(nb):
            if run[b] is None:
                continue
            i, tr, end = run[b]
            tr.add(ctx.diag(b)["free_energy"])
            if tr.n >= end or (horizons is None and tr.conv is not None):
                finish(b, True)
                start(b)
        if time.time() - last > 30:
            last = time.time()
            log("  %s: %d/%d done, %d running, %.0f s" % (label, sum(r is not None for r in results), len(cases),
                                                         sum(r is not None for r in run), time.time() - t0))
    ctx.close()
    log("  %s: %d cases in %.0f s" % (label, len(cases), time.time() - t0))
    return results


def steps_to_band(F, Fstar, end_step):
    """First sampled step after which |F - F*| <= BAND |F*| holds up to
    end_step; None if the sample at end_step is outside the band."""
    k_end = end_step // EVERY
    if len(F) <= k_end:
        return None
    err = np.abs(F[:k_end + 1] - Fstar) / abs(Fstar)
    ok = np.isfinite(err) & (err <= BAND)
    if not ok[-1]:
        return None
    bad = np.nonzero(~ok)[0]
    return 0 if len(bad) == 0 else int(bad[-1] + 1) * EVERY


def q_error(Q, Qstar, fluid):
    """Mean over fluid sites of |Q - Q*|_F^2 (5-component storage expanded)."""
    d = Q - Qstar
    w = np.array([1.0, 2.0, 2.0, 1.0, 2.0])
    sq = np.tensordot(w, d * d, axes=1) + (d[0] + d[3]) ** 2
    return float((sq * fluid).sum() / fluid.sum())


def save_weights(net, path):
    """Weights in the library's file format (lc_nn_save)."""
    net.save(path)


def load_weights(net, path):
    net.load(path)


def relaxed_states(cases, L, cap, batch, hydro, tile, label):
    """Plain relaxations of the cases on a pool of ``batch`` boxes: the
    relaxed Q (FP64 host arrays), F samples and convergence steps."""
    res = stream(cases, L, cap, batch, hydro, tile, label)
    return [dict(c, Q=r["Q"], F=r["F"], conv=r["conv"]) for c, r in zip(cases, res)]


def prediction_error(net, d, L):
    Q = helix(d, L) + Q_EQ * net.predict(nn_case(d, L))
    return q_error(Q, d["Q"], fluid_mask(d, L))


def train(net, data, L, epochs, lr0, lr1, seed, held=()):
    """Adam on one case per step, cosine learning-rate decay lr0 -> lr1."""
    fluid = fluid_masks(data, L)
    total = epochs * len(data)
    hist = []
    it = 0
    for ep in range(epochs):
        order = np.argsort(inputs.uniform(seed, len(data), stream=100 + ep))
        losses = []
        for j in order:
            lr = lr1 + 0.5 * (lr0 - lr1) * (1 + math.cos(math.pi * it / total))
            losses.append(net.train_step(nn_case(data[j], L), data[j]["Q"], fluid[j], lr))
            it += 1
        rec = {"epoch": ep, "train_loss": float(np.mean(losses))}
        if held:
            rec["held_loss"] = float(np.mean([prediction_error(net, d, L) for d in held]))
        hist.append(rec)
        log("  epoch %d: train loss %.4e%s" % (ep, rec["train_loss"],
                                             ", held-out %.4e" % rec["held_loss"] if held else ""))
    return hist


def compare(net, held, L, cap, hydro, tile, batch):
    """Warm runs of the held-out cases against their plain relaxations, each
    warm run as long as its plain run took to converge (cap if it did not)."""
    horizons = [d["conv"] if d["conv"] is not None else cap for d in held]
    warm = stream(held, L, cap, batch, hydro, tile, "warm", net=net, horizons=horizons, keep_Q=False)
    rows = []
    for d, w in zip(held, warm):
        row = {k: d[k] for k in ("seed", "a", "pitch", "anchoring", "conv")}
        row["q_err_helix"] = q_error(helix(d, L), d["Q"], fluid_mask(d, L))
        row["q_err_warm"] = prediction_error(net, d, L)
        row["F_plain"] = d["F"].tolist()
        row["F_warm"] = w["F"].tolist()
        if d["conv"] is not None:
            Fstar = d["F"][d["conv"] // EVERY]
            n_plain = steps_to_band(d["F"], Fstar, d["conv"])
            n_warm = steps_to_band(w["F"], Fstar, d["conv"]) if w["ok"] else None
            row.update(F_star=float(Fstar), n_plain=n_plain, n_warm=n_warm, fallback=n_warm is None,
                       n_warm_charged=(n_warm if n_warm is not None else d["conv"] + n_plain),
                       err0_plain=float(abs(d["F"][0] - Fstar) / abs(Fstar)),
                       err0_warm=float(abs(w["F"][0] - Fstar) / abs(Fstar)))
        rows.append(row)
        log("  seed %d a %.2f p %.2f %s: plain %s warm %s%s (Q err helix %.3e warm %.3e)" % (
            d["seed"], d["a"], d["pitch"], d["anchoring"], row.get("n_plain"), row.get("n_warm"),
            " FALLBACK" if row.get("fallback") else "", row["q_err_helix"], row["q_err_warm"]))
    return rows


def summary(rows):
    ev = [r for r in rows if r.get("n_plain") is not None]
    if not ev:
        return {"evaluated": 0, "not_converged": len(rows)}
    plain = np.array([r["n_plain"] for r in ev], float)
    warm = np.array([r["n_warm_charged"] for r in ev], float)
    return {"evaluated": len(ev), "not_converged": len(rows) - len(ev),
            "fallbacks": int(sum(r["fallback"] for r in ev)),
            "plain_steps_mean": float(plain.mean()), "warm_steps_mean": float(warm.mean()),
            "ratio_of_means": float(warm.sum() / max(plain.sum(), 1.0)),
            "warm_faster": int((warm < plain).sum()), "warm_slower": int((warm > plain).sum()),
            "q_err_helix_mean": float(np.mean([r["q_err_helix"] for r in ev])),
            "q_err_warm_mean": float(np.mean([r["q_err_warm"] for r in ev]))}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    for name in ("train", "evaluate"):
        p = sub.add_parser(name)
        p.add_argument("--out", required=True)
        p.add_argument("--L", type=int, default=64)
        p.add_argument("--hydro", type=int, default=0)
        p.add_argument("--batch", type=int, default=32)
        p.add_argument("--weights", default=None)
        p.add_argument("--nheld", type=int, default=16)
        p.add_argument("--held-cap", type=int, default=120000)
    tr = sub.choices["train"]
    tr.add_argument("--ntrain", type=int, default=256)
    tr.add_argument("--seed0", type=int, default=TRAIN_SEED0)
    tr.add_argument("--cap", type=int, default=50000)
    tr.add_argument("--epochs", type=int, default=40)
    tr.add_argument("--lr0", type=float, default=1e-3)
    tr.add_argument("--lr1", type=float, default=2e-5)
    tr.add_argument("--net-seed", type=int, default=1)
    tr.add_argument("--out-scale", type=float, default=0.01,
                    help="scale of the output layer's initial weights (the untrained net then predicts ~0)")
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    L = args.L
    tile, times = pick_tile(min(args.batch, 32), L, args.hydro)
    log("tile %d, step ms per tile %s" % (tile, {k: round(v, 4) for k, v in times.items()}))
    net = nn.Net(L, seed=getattr(args, "net_seed", 1))
    if args.weights:
        load_weights(net, args.weights)
    elif args.cmd == "train":
        W, b = net.get_layer(3)
        net.set_layer(3, W * args.out_scale, 0 * b)
    held = []
    if args.nheld > 0:
        cases = [inputs.warmstart_case(s) for s in range(HELD_SEED0, HELD_SEED0 + args.nheld)]
        held = relaxed_states(cases, L, args.held_cap, args.batch, args.hydro, tile, "plain")
    info = {"args": vars(args), "tile": tile, "params": PARAMS}
    if args.cmd == "train":
        t0 = time.time()
        cases = [inputs.warmstart_case(s) for s in range(args.seed0, args.seed0 + args.ntrain)]
        data = relaxed_states(cases, L, args.cap, args.batch, args.hydro, tile, "data")
        info["gen_seconds"] = time.time() - t0
        log("generated %d states in %.0f s" % (len(data), info["gen_seconds"]))
        t0 = time.time()
        info["history"] = train(net, data, L, args.epochs, args.lr0, args.lr1, args.seed0,
                                [d for d in held if d["conv"] is not None])
        info["train_seconds"] = time.time() - t0
        save_weights(net, os.path.join(args.out, "weights.lcnn"))
        info["nn_time_ms"] = net.time(nn_case(data[0], L), data[0]["Q"], fluid_mask(data[0], L), n=20)
        info["cases"] = [{k: d[k] for k in ("seed", "a", "pitch", "anchoring", "conv")} for d in data]
        log("trained in %.0f s; %s" % (info["train_seconds"], info["nn_time_ms"]))
        with open(os.path.join(args.out, "train_only.json"), "w") as f:
            json.dump(info, f, indent=1)
    if held:
        rows = compare(net, held, L, args.held_cap, args.hydro, tile, args.batch)
        info["summary"] = summary(rows)
        info["rows"] = rows
        log("summary %s" % json.dumps(info["summary"]))
    with open(os.path.join(args.out, "%s.json" % args.cmd), "w") as f:
        json.dump(info, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
