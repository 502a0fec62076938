"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the oracle.

This module holds initial conditions and workload descriptions only; it
contains none of the method's arithmetic and imports nothing else from the
package.  Arrays are float64, structure-of-arrays ``[component, z, y, x]``,
Q components ordered (xx, xy, xz, yy, yz).

Random numbers come from splitmix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) keyed by (seed, site,
component), so any sub-block of a field can be regenerated independently.
"""
import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(keys: np.ndarray) -> np.ndarray:
    """splitmix64 output for each uint64 state value in ``keys``."""
    with np.errstate(over="ignore"):
        z = keys.astype(np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, n: int, stream: int = 0) -> np.ndarray:
    """n uniform doubles in [0, 1) for counter values 0..n-1 of (seed, stream)."""
    with np.errstate(over="ignore"):
        base = np.uint64(seed) * np.uint64(0xD1B54A32D192ED03) + np.uint64(stream) * _GOLDEN
        keys = base + np.arange(n, dtype=np.uint64)
    bits = splitmix64(keys) >> np.uint64(11)
    return bits.astype(np.float64) * (1.0 / 9007199254740992.0)


def uniaxial_q(nx, ny, nz, amplitude, director=(0.0, 0.0, 1.0)):
    """Uniform uniaxial Q = amplitude (n n - I/3) (paper convention)."""
    n = np.asarray(director, dtype=np.float64)
    n = n / np.linalg.norm(n)
    comp = [n[0] * n[0] - 1.0 / 3.0, n[0] * n[1], n[0] * n[2], n[1] * n[1] - 1.0 / 3.0, n[1] * n[2]]
    Q = np.empty((5, nz, ny, nx))
    for c in range(5):
        Q[c] = amplitude * comp[c]
    return Q


def noisy_nematic_q(nx, ny, nz, amplitude, seed, noise=1e-3, director=(0.0, 0.0, 1.0)):
    """Uniaxial Q plus independent U(-noise, +noise) on each stored component.

    The noise for (site s, component c) is counter 5*s + c of the seed's stream.
    """
    Q = uniaxial_q(nx, ny, nz, amplitude, director)
    N = nx * ny * nz
    r = uniform(seed, 5 * N).reshape(N, 5).T.reshape(5, nz, ny, nx)
    return Q + noise * (2.0 * r - 1.0)


def helix_q(nx, ny, nz, q0, amplitude):
    """Cholesteric helix along z: n(z) = (cos q0 z, sin q0 z, 0), z the site index."""
    z = np.arange(nz, dtype=np.float64)
    c, s = np.cos(q0 * z), np.sin(q0 * z)
    Q = np.empty((5, nz, ny, nx))
    Q[0] = amplitude * (c * c - 1.0 / 3.0)[:, None, None]
    Q[1] = amplitude * (c * s)[:, None, None]
    Q[2] = 0.0
    Q[3] = amplitude * (s * s - 1.0 / 3.0)[:, None, None]
    Q[4] = 0.0
    return Q


def commensurate_pitch(L, p):
    """Pitch snapped so that the box holds a whole number of half pitches."""
    k = max(1, int(round(2.0 * L / p)))
    return 2.0 * L / k


def batch_boxes(seed, nbox=48, sizes=(32, 40, 48, 56, 64), a_range=(3.0, 12.0),
                p_range=(16.0, 48.0)):
    """Seeded sweep of cubic cholesteric boxes: (L, a, pitch) per box."""
    r = uniform(seed, 3 * nbox, stream=7).reshape(nbox, 3)
    out = []
    for b in range(nbox):
        L = sizes[min(len(sizes) - 1, int(r[b, 0] * len(sizes)))]
        a = a_range[0] + (a_range[1] - a_range[0]) * r[b, 1]
        a = min(a, 0.5 * L - 3.0)
        p = commensurate_pitch(L, p_range[0] + (p_range[1] - p_range[0]) * r[b, 2])
        out.append({"L": L, "a": a, "pitch": p, "q0": 2.0 * math.pi / p})
    return out


# Warm-start cases on a 64^3 box: pitches 128/k, each a whole number of half
# pitches in the box.
WARM_PITCHES = tuple(128.0 / k for k in (8, 7, 6, 5, 4, 3))


def warmstart_case(seed, a_range=(3.0, 12.0)):
    """One seeded warm-start case: radius ~ U[a_range], pitch drawn from
    WARM_PITCHES, normal or planar anchoring with equal odds."""
    r = uniform(seed, 3, stream=11)
    a = a_range[0] + (a_range[1] - a_range[0]) * r[0]
    p = WARM_PITCHES[min(len(WARM_PITCHES) - 1, int(r[1] * len(WARM_PITCHES)))]
    return {"seed": int(seed), "a": float(a), "pitch": float(p), "anchoring": "normal" if r[2] < 0.5 else "planar"}


# Material and LB parameters of the synthetic workloads (lattice units).
NEMATIC = dict(tau=1.0, rho0=1.0, A0=0.01, gamma=3.0, K=0.01, q0=0.0, xi=0.7, Gamma=0.5)

# Material parameters of the paper's cholesteric study (Sec. 3): A0 = 1,
# K = 0.065, gamma = 3 (tau = 0), xi = 0.7, Gamma = 0.5; chirality 0.3 at
# pitch 32.
PAPER_CHOLESTERIC = dict(tau=1.0, rho0=1.0, A0=1.0, gamma=3.0, K=0.065, q0=0.0, xi=0.7, Gamma=0.5)

# Uniaxial amplitude for S = 0.33 in the convention Q = (S/2)(3nn - I),
# i.e. q = 1.5 S in the paper's Q = q(nn - I/3).
Q_INIT = 1.5 * 0.33

WORKLOADS = {
    "nematic32_fp64": dict(L=32, precision="fp64", params=NEMATIC, a=4.0, anchoring="planar",
                           W=0.01, S0=0.5, seed=1, steps=200),
    "drag128_fp32": dict(L=128, precision="fp32", params=NEMATIC, a=8.0, anchoring="normal",
                         W=0.01, S0=0.5, seeds=(2, 3), speed=1e-3, steps=5000),
    "cholesteric128_fp32": dict(L=128, precision="fp32", params=dict(NEMATIC, q0=2 * math.pi / 32),
                                radii=(4.0, 8.0, 12.0, 16.0), anchoring="normal", W=math.inf,
                                S0=0.5, seeds=(10, 11, 12, 13), steps=10000),
}
