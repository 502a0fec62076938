"""Host-side logic of the warm-start pipeline (no GPU): case generator,
convergence bookkeeping, steps-to-relax, the Q error measure and the
weights file round trip."""
import math

import numpy as np
import pytest

from paper_1102_2193_amd import inputs
from paper_1102_2193_amd import warmstart as ws


def test_cases_are_seeded_and_in_range():
    cs = [inputs.warmstart_case(5000 + i) for i in range(300)]
    assert cs[7] == inputs.warmstart_case(5007)
    assert all(3.0 <= c["a"] <= 12.0 for c in cs)
    assert {c["pitch"] for c in cs} == set(inputs.WARM_PITCHES)
    assert {c["anchoring"] for c in cs} == {"normal", "planar"}
    # every pitch holds a whole number of half pitches in a 64 box
    for p in inputs.WARM_PITCHES:
        assert 2 * 64 / p == pytest.approx(round(2 * 64 / p), abs=1e-12)


class _FakeContext:
    """Stands in for a context: F of box b at step n is seq[b](n)."""

    def __init__(self, seq):
        self.seq, self.n = seq, 0

    def set_Q(self, b, q):
        pass

    def step(self, n):
        self.n += n

    def diag(self, b):
        return {"free_energy": self.seq[b](self.n)}


def test_convergence_must_hold_for_the_whole_window(monkeypatch):
    decay = lambda n: -1000.0 - math.exp(-n / 2000.0)
    wobble = lambda n: -1000.0 - 0.01 * math.sin(n / 3000.0)   # turning points pass a single-window test
    monkeypatch.setattr(ws, "make_context", lambda cases, L, hydro, tile: _FakeContext([decay, wobble]))
    monkeypatch.setattr(ws, "helix", lambda c, L: None)
    _, F, conv, ok = ws.relax([{}, {}], cap=60000)
    assert ok and len(F[0]) == 60000 // ws.EVERY + 1
    # |F(n) - F(n-1000)| = e^{-n/2000} (e^{1/2} - 1) < 1e-7 * 1000 first at
    # n = 17557.8..., i.e. the sample at 17600; held for 4000 more steps
    assert conv[0] == 21600
    assert conv[1] is None


class _FakePool:
    """A context whose box b follows F = seq(case)(steps since its case was
    set); the case is identified by its radius."""

    def __init__(self, seqs):
        self.seqs, self.case, self.n, self.closed = seqs, {}, {}, False

    def set_colloid(self, b, pos, a, **kw):
        self.case[b] = a

    def set_Q(self, b, q):
        self.n[b] = 0

    def step(self, n):
        for b in self.n:
            self.n[b] += n

    def diag(self, b):
        return {"free_energy": self.seqs[self.case[b]](self.n[b])}

    def get_Q(self, b):
        return np.full(2, self.case[b])

    def close(self):
        self.closed = True


def test_box_counts_follow_the_case_mix():
    assert ws.box_counts([16.0] * 30 + [32.0] * 10, 8) == {16.0: 6, 32.0: 2}
    assert ws.box_counts([16.0] * 3 + [32.0] * 1, 32) == {16.0: 3, 32.0: 1}   # never more boxes than cases
    c = ws.box_counts([16.0] * 50 + [21.0] + [32.0] * 49, 6)
    assert c[21.0] == 1 and sum(c.values()) == 6


def test_streamed_runs_equal_runs_alone(monkeypatch):
    """Each case's samples and convergence step in a pool of two boxes (boxes
    taking new cases as runs end) equal those of the case run alone."""
    seqs = {float(k): (lambda k: lambda n: -1000.0 - math.exp(-n / (800.0 * k)))(k) for k in range(1, 8)}
    seqs[9.0] = lambda n: -1000.0 - 0.01 * math.sin(n / 3000.0)   # never converges: runs to the cap
    cases = [{"a": a, "pitch": 16.0 if a % 2 else 32.0, "anchoring": "normal"} for a in sorted(seqs)]
    monkeypatch.setattr(ws, "make_context", lambda cs, L, hydro, tile: _FakePool(seqs))
    monkeypatch.setattr(ws, "helix", lambda c, L: None)
    res = ws.stream(cases, 8, 30000, 2, 0, None, "test")
    for c, r in zip(cases, res):
        alone = _FakeContext([seqs[c["a"]]])
        monkeypatch.setattr(ws, "make_context", lambda cs, L, hydro, tile: alone)
        _, F, conv, ok = ws.relax([c], cap=30000)
        assert r["ok"] and r["conv"] == conv[0]
        np.testing.assert_array_equal(r["F"], F[0])
        assert r["Q"][0] == c["a"]
    assert res[-1]["conv"] is None and len(res[-1]["F"]) == 30000 // ws.EVERY + 1
    # horizons: each run stops at its own horizon
    monkeypatch.setattr(ws, "make_context", lambda cs, L, hydro, tile: _FakePool(seqs))
    hz = [1000 * (i + 1) for i in range(len(cases))]
    res = ws.stream(cases, 8, 30000, 3, 0, None, "test", net=None, horizons=hz, keep_Q=False)
    assert [len(r["F"]) - 1 for r in res] == [h // ws.EVERY for h in hz]


def test_steps_to_band():
    E = ws.EVERY
    F = np.array([10, 5, 2, 1.0002, 1.00005, 0.99999, 1.00001, 1.0])
    assert ws.steps_to_band(F, 1.0, 7 * E) == 4 * E
    assert ws.steps_to_band(F, 1.0, 5 * E) == 4 * E
    assert ws.steps_to_band(np.array([1.0, 1.0]), 1.0, E) == 0
    # outside the band at the end: a different minimum, i.e. a fallback
    assert ws.steps_to_band(np.array([10, 1.0, 1.5]), 1.0, 2 * E) is None
    assert ws.steps_to_band(np.array([10, 1.0, np.nan]), 1.0, 2 * E) is None


def test_q_error_is_the_full_tensor_frobenius_norm():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(5, 3, 2, 2))
    xx, xy, xz, yy, yz = d
    M = np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, -xx - yy]])
    fluid = np.ones((3, 2, 2), np.uint8)
    fluid[0, 0, 0] = 0
    ref = ((M ** 2).sum(axis=(0, 1)) * fluid).sum() / fluid.sum()
    assert ws.q_error(d, 0 * d, fluid) == pytest.approx(ref, rel=1e-14)


def test_summary_charges_fallbacks():
    rows = [{"n_plain": 1000, "n_warm_charged": 100, "fallback": False, "q_err_helix": 1e-2, "q_err_warm": 1e-3},
            {"n_plain": 500, "n_warm_charged": 9500, "fallback": True, "q_err_helix": 1e-2, "q_err_warm": 1e-3},
            {"conv": None, "q_err_helix": 1e-2, "q_err_warm": 1e-3}]
    s = ws.summary(rows)
    assert s["evaluated"] == 2 and s["not_converged"] == 1 and s["fallbacks"] == 1
    assert s["ratio_of_means"] == pytest.approx(9600 / 1500)
    assert s["warm_faster"] == 1 and s["warm_slower"] == 1


def read_weight_file(path):
    """Parse the weight file format documented for lc_nn_save."""
    raw = open(path, "rb").read()
    assert raw[:8] == b"LCNNWTS1"
    version, nl = np.frombuffer(raw, np.int32, 2, 8)
    assert version == 1 and nl == 4
    off, layers = 16, []
    for _ in range(nl):
        cout, cin, taps, pad = np.frombuffer(raw, np.int32, 4, off)
        off += 16
        W = np.frombuffer(raw, np.float32, cout * cin * taps, off).reshape(cout, cin, taps)
        off += W.nbytes
        b = np.frombuffer(raw, np.float32, cout, off)
        off += b.nbytes
        layers.append((W, b))
    assert off == len(raw)
    return layers


def test_committed_weights_have_the_network_shapes():
    from paper_1102_2193_amd import nn
    for l, (W, b) in enumerate(read_weight_file(ws.WEIGHTS)):
        assert W.shape == (nn.COUT[l], nn.CIN[l], 27)
        assert b.shape == (nn.COUT[l],)
        assert np.all(np.isfinite(W)) and np.all(np.isfinite(b))
