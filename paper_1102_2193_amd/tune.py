"""Tile-shape autotuner for the fused kernel.

Every tile shape computes the same per-site arithmetic (the parity tests
check that); the shapes differ only in LDS footprint, halo overhead and
occupancy.  The tuner times each shape with HIP events on the live context
and keeps the fastest in a JSON cache keyed by the batch's box sizes,
precision and a hash of the kernel and runtime sources, so that a choice
measured on other kernels is never reused.  Tuning on a live context
advances its state by the timed steps.
"""
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")
SOURCES = ("lc_kernels.hip", "lc_kernels.hpp", "lc_dev.hpp", "lc_march.hpp", "lc_arch.hpp", "lc_reduce.hpp",
           "lc_runtime.hip")


def sources_hash():
    """First 16 hex digits of the SHA-256 of the sources that decide a
    tile's speed (kernels, device definitions, work schedule)."""
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def batch_key(ctx):
    dims = ",".join("%dx%dx%d" % (p.nx, p.ny, p.nz) for p in ctx.box_params)
    prec = "fp64" if ctx.box_params[0].precision == 1 else "fp32"
    if len(dims) > 200:
        dims = "n%d-%s" % (len(ctx.box_params), hashlib.sha1(dims.encode()).hexdigest()[:16])
    return "%s:%s:%s" % (prec, dims, sources_hash())


def load_cache():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(ctx, steps=40, warm=8):
    """Time every tile shape on ctx; returns {tile_id: mean step ms}."""
    from . import lc
    res = {}
    for t in range(ctx.num_tiles()):
        try:
            ctx.set_tile(t)
        except lc.LCError:     # a shape the context's boxes cannot use
            continue
        ctx.time_kernel(warm)
        res[t] = ctx.time_kernel(steps)["step_ms"]
    return res


def best_tile(ctx, name="", save=True):
    key = batch_key(ctx)
    cache = load_cache()
    if key in cache:
        return int(cache[key]["tile"])
    res = tune(ctx)
    best = min(res, key=res.get)
    if save:
        cache[key] = {"tile": best, "shape": list(ctx.tile_shape(best)), "step_ms": res,
                      "workload": name}
        try:
            with open(CACHE, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return best
