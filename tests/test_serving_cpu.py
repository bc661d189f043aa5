"""Serving logic without a GPU: the seeded request trace and the server's
admission/retirement loop driven by a stand-in executor."""
import numpy as np
import pytest

from paper_1704_03172_amd import inputs


def test_trace_is_seeded_and_shaped():
    a = inputs.serving_trace(300, 50.0, seed=4)
    b = inputs.serving_trace(300, 50.0, seed=4)
    assert [r["n"] for r in a] == [r["n"] for r in b]
    assert [r["arrival"] for r in a] == [r["arrival"] for r in b]
    ns = {r["n"] for r in a}
    assert ns <= set(range(256, 4097, 256)) and len(ns) >= 12
    assert all(1000 <= r["nsteps"] <= 4000 for r in a)
    gaps = np.diff([0.0] + [r["arrival"] for r in a])
    assert 0.015 < gaps.mean() < 0.025                   # mean rate ~ 50 / s
    for r in a:
        L = r["sponge"]
        assert L == min(64, r["n"] // 8)
        assert L <= r["src"][0] < r["n"] - L and r["src"][1] == L
        assert 3 <= len(r["speeds"]) <= 8 and 1 <= len(r["blobs"]) <= 5


@pytest.mark.parametrize("k", [0, 5, 17])
def test_medium_in_range(k):
    req = inputs.serving_trace(20, 50.0, seed=4, sizes=[256, 512])[k]
    c = inputs.serving_speed_numpy(req)
    assert c.shape == (req["n"], req["n"])
    assert c.min() >= 0.3 * 0.9 - 1e-12 and c.max() <= 0.57 * 1.1 + 1e-12
    assert (c * c).max() < 0.5                            # D2Q5 c^2 limit
    rec = inputs.serving_receivers(req)
    assert rec.shape == (128, 2) and rec[:, 0].min() >= 0 and rec[:, 0].max() < req["n"]


def test_torch_medium_matches_numpy():
    torch = pytest.importorskip("torch")
    req = inputs.serving_trace(3, 50.0, seed=9, sizes=[256])[1]
    a = inputs.serving_speed_numpy(req)
    b = inputs.serving_speed_torch(req, "cpu").numpy()
    np.testing.assert_allclose(a, b, rtol=1e-13)


class FakeBatch:
    """Executor stand-in: advances shot times by k per tick."""

    def __init__(self, max_shots):
        import torch
        self.device = torch.device("cpu")
        self.max_shots = max_shots
        self.t = {}
        self.end = {}
        self.adds = []
        self.peak = 0

    def shot_bytes(self, desc):
        return 44 * desc.nx * desc.ny + 8 * (desc.nsteps + 1)

    def add(self, desc, c2, w, rec):
        import torch
        slot = min(set(range(self.max_shots)) - set(self.t))
        self.t[slot] = 0
        self.end[slot] = desc.nsteps
        self.adds.append(desc.nx)
        self.peak = max(self.peak, len(self.t))
        assert c2.shape == (desc.ny, desc.nx) and len(w) == desc.nsteps + 1
        return slot

    def tick(self, k):
        for s in self.t:
            self.t[s] = min(self.t[s] + k, self.end[s])

    def times(self):
        out = np.full(self.max_shots, -1, dtype=np.int64)
        for s, v in self.t.items():
            out[s] = v
        return out

    def completed(self):   # ticks complete at once
        return self.times()

    def in_flight(self):
        return 0

    def wait_oldest(self):
        return False

    def remove(self, slot):
        import torch
        del self.t[slot]
        del self.end[slot]
        return torch.zeros((1, 2))

    def close(self):
        pass


def test_server_admission_and_completion():
    pytest.importorskip("torch")
    from paper_1704_03172_amd import lbwave, serve
    try:
        lbwave.lib()
    except RuntimeError:
        pytest.skip("library not built")
    trace = inputs.serving_trace(12, 1e6, seed=4, sizes=[256, 512], steps=(100, 400))
    fb = FakeBatch(3)
    srv = serve.ShotServer(budget_bytes=44 * 512 * 512 * 2 + 10000, max_slots=3, tick_steps=50, batch=fb,
                           policy="fifo")
    recs, summary = srv.run(trace)
    assert summary["completed"] == 12
    assert fb.peak <= 3
    assert fb.adds == [r["n"] for r in sorted(trace, key=lambda r: r["arrival"])]   # FIFO admission
    for r in recs:
        assert r["arrival"] <= r["admit"] <= r["done"]
    assert summary["latency_p99_s"] >= summary["latency_p50_s"] >= 0


def test_summary_math():
    from paper_1704_03172_amd import serve
    recs = [{"arrival": 0.0, "admit": 1.0, "done": 3.0, "n": 100, "nsteps": 10},
            {"arrival": 1.0, "admit": 1.0, "done": 2.0, "n": 200, "nsteps": 5}]
    s = serve.summarize(recs, 3.0)
    assert s["completed"] == 2 and abs(s["shots_per_s"] - 2 / 3) < 1e-3
    assert abs(s["GLUPS"] - (100 * 100 * 10 + 200 * 200 * 5) / 3.0 / 1e9) < 1e-6
    assert s["latency_p50_s"] == pytest.approx(2.0)


def test_server_sjf_and_node_cap():
    pytest.importorskip("torch")
    from paper_1704_03172_amd import lbwave, serve
    try:
        lbwave.lib()
    except RuntimeError:
        pytest.skip("library not built")
    trace = inputs.serving_trace(10, 1e6, seed=5, sizes=[256, 512, 768], steps=(100, 300))
    fb = FakeBatch(8)
    srv = serve.ShotServer(budget_bytes=1 << 40, max_slots=8, tick_steps=40, batch=fb,
                           policy="sjf", node_cap=768 * 768)
    recs, summary = srv.run(trace)
    assert summary["completed"] == 10
    # the node cap admits one 768^2 shot at a time, or several smaller ones
    assert fb.peak <= 9
    order = sorted(trace, key=lambda r: (r["n"] ** 2 * r["nsteps"], r["arrival"]))
    assert fb.adds[0] == order[0]["n"]          # all arrived at once: shortest first


def test_sjf_aging_orders_long_waiters_first():
    """With aging, a large request that has waited long goes before fresh
    small ones; without waiting the order is shortest first."""
    from paper_1704_03172_amd import serve
    big = {"n": 4096, "nsteps": 4000, "arrival": 0.0}
    small = {"n": 256, "nsteps": 1000, "arrival": 9.9}
    rate = 4e11
    s_big = 4096 * 4096 * 4000 / rate
    assert serve._pick_order([big, small], "sjf", 0.0, rate, 0.05)[0] is small     # waits equal (none)
    assert serve._pick_order([big, small], "sjf", 10.0, rate, 0.05)[0] is big       # waited 10 s
    assert serve._pick_order([big, small], "sjf", 10.0, rate, 0.0)[0] is small      # no aging: starves
    assert serve._pick_order([big, small], "fifo", 10.0, rate, 0.05)[0] is big
    assert s_big - 0.05 * 10.0 < 0
