"""Scheduling logic of the serving loop on the CPU, with a stand-in executor:
session/round validation (stale rounds rejected), admission by HBM budget,
LRU eviction of idle key sets, batching of waiting requests across clients,
and continuous batching (arrivals join later launches while others run)."""
import itertools

import numpy as np
import pytest

from paper_2509_01253_amd.serving import Request, Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Batches complete `dur` seconds of fake time after launch."""

    def __init__(self, clock, key_bytes=100, io_per_req=10, ws_per_req=5, dur=1.0):
        self.clock = clock
        self.kb, self.io, self.ws_per, self.dur = key_bytes, io_per_req, ws_per_req, dur
        self.loaded = {}
        self.ws = {}
        self.launches = []
        self.loads = []

    def has_layer(self, layer):
        return layer in ("fc", "conv")

    def layer_params(self, layer):
        return "N16" if layer == "fc" else "N15"

    def library_bytes(self):
        return sum(self.loaded.values()) + sum(self.ws.values())

    def key_bytes(self, client, params):
        return self.kb

    def io_bytes(self, layer, batch):
        return self.io * len(batch)

    def workspace_growth(self, layer, n, stream):
        return max(0, self.ws_per * n - self.ws.get(stream, 0))

    def load_keys(self, client, params, stream):
        h = (client, params, len(self.loads))
        self.loads.append(h)
        self.loaded[h] = self.kb
        return h

    def release_keys(self, h):
        del self.loaded[h]

    def launch(self, layer, batch, handles, stream):
        self.ws[stream] = max(self.ws.get(stream, 0), self.ws_per * len(batch))
        self.launches.append((layer, [r.rid for r in batch], self.clock()))
        return (self.clock() + self.dur,), None, self.io * len(batch)

    def done(self, token):
        return self.clock() >= token[0]

    def collect(self, token, out, reqs):
        return [(("y", r.rid), r.level - 1) for r in reqs]


def _req(rid, client, rnd=1, layer="fc", level=5):
    return Request(rid, client, f"s-{client}", rnd, layer, level, x=None)


def test_session_rounds():
    clk = FakeClock()
    srv = Server(FakeExecutor(clk), hbm_budget=10 ** 6, clock=clk)
    srv.open_session("s-a", "a")
    assert srv.submit(_req(1, "a", 1))
    assert not srv.submit(_req(2, "a", 1))          # replayed round
    assert not srv.submit(_req(3, "a", 3))          # skipped round
    assert srv.submit(_req(4, "a", 2))
    assert not srv.submit(_req(5, "b", 1))          # unknown session
    assert not srv.submit(Request(6, "b", "s-a", 3, "fc", 5, None))  # other client's session
    assert not srv.submit(Request(7, "a", "s-a", 3, "nope", 5, None))
    assert srv.rejected == 5
    assert "stale" in srv.results[2].status


def test_batches_across_clients_and_levels():
    clk = FakeClock()
    ex = FakeExecutor(clk)
    srv = Server(ex, hbm_budget=10 ** 6, streams=2, max_batch=3, clock=clk)
    for c in "abcde":
        srv.open_session(f"s-{c}", c)
    for i, c in enumerate("abcde"):
        srv.submit(_req(i, c, level=4 + i))
    srv.submit(_req(10, "a", 2, layer="conv"))
    srv.pump()
    # oldest request's layer first, up to max_batch, mixing clients and levels
    assert ex.launches[0][1] == [0, 1, 2]
    assert ex.launches[1][1] == [3, 4]
    assert len(srv.queue) == 1
    clk.t = 1.0
    srv.pump()
    assert ex.launches[2][1] == [10]
    clk.t = 2.0
    srv.pump()
    assert all(srv.results[r].status == "ok" for r in (0, 1, 2, 3, 4, 10))
    assert srv.results[3].y == ("y", 3) and srv.results[3].level == 6


def test_continuous_batching_admits_arrivals_while_running():
    clk = FakeClock()
    ex = FakeExecutor(clk, dur=1.0)
    srv = Server(ex, hbm_budget=10 ** 6, streams=2, clock=clk, overlap_min_queue=1)
    for c in "abc":
        srv.open_session(f"s-{c}", c)
    srv.submit(_req(0, "a"))
    srv.pump()                      # batch 1 on stream 0
    clk.t = 0.3
    srv.submit(_req(1, "b"))
    srv.pump()                      # joins immediately on the free stream 1
    clk.t = 0.5
    r2 = _req(2, "c")
    r2.arrival = clk.t
    srv.submit(r2)
    srv.pump()                      # both streams busy: waits
    assert [l[1] for l in ex.launches] == [[0], [1]]
    clk.t = 1.0
    srv.pump()                      # stream 0 frees -> request 2 starts at t = 1.0
    assert ex.launches[2] == ("fc", [2], 1.0)
    clk.t = 2.0
    srv.pump()
    assert srv.results[2].latency == 1.5


def test_lone_request_waits_instead_of_overlapping():
    """With the default overlap threshold a single waiting request does not start a
    second batch beside a running one; two waiting requests do."""
    clk = FakeClock()
    ex = FakeExecutor(clk, dur=1.0)
    srv = Server(ex, hbm_budget=10 ** 6, streams=2, clock=clk)
    for c in "abcd":
        srv.open_session(f"s-{c}", c)
    srv.submit(_req(0, "a"))
    srv.pump()                      # batch 1 on stream 0
    clk.t = 0.3
    srv.submit(_req(1, "b"))
    srv.pump()                      # alone in the queue: waits for stream 0
    assert [l[1] for l in ex.launches] == [[0]]
    clk.t = 0.4
    srv.submit(_req(2, "c", layer="conv"))
    srv.pump()                      # two waiting: a second batch starts on stream 1
    assert [l[1] for l in ex.launches] == [[0], [1]]
    assert srv.max_inflight == 2
    clk.t = 1.0
    srv.pump()                      # stream 0 frees, stream 1 still runs: the lone conv request waits
    assert len(ex.launches) == 2
    clk.t = 1.4
    srv.pump()                      # nothing in flight -> it starts
    assert ex.launches[2] == ("conv", [2], 1.4)


def test_admission_by_budget_and_lru_eviction():
    clk = FakeClock()
    # budget: two key sets (200) + io/workspace of a single request (15) fit; three key sets do not
    ex = FakeExecutor(clk, key_bytes=100, io_per_req=10, ws_per_req=5)
    srv = Server(ex, hbm_budget=230, streams=1, clock=clk)
    for c in "abc":
        srv.open_session(f"s-{c}", c)
    srv.submit(_req(0, "a"))
    srv.pump()
    clk.t = 1.0
    srv.pump()
    srv.submit(_req(1, "b", layer="fc"))
    srv.pump()
    clk.t = 2.0
    srv.pump()
    assert len(ex.loaded) == 2
    srv.submit(_req(2, "c"))
    srv.pump()                      # needs a third key set: the LRU idle one (a) is evicted
    assert srv.evictions == 1
    assert ("a", "N16", 0) not in ex.loaded
    clk.t = 3.0
    srv.pump()
    srv.submit(_req(3, "a", 2))     # a comes back: its keys are uploaded again
    srv.pump()
    assert len(ex.loads) == 4 and srv.evictions == 2


def test_waits_when_nothing_can_be_evicted():
    clk = FakeClock()
    ex = FakeExecutor(clk, key_bytes=100, io_per_req=10, ws_per_req=5)
    srv = Server(ex, hbm_budget=130, streams=2, clock=clk)
    for c in "ab":
        srv.open_session(f"s-{c}", c)
    srv.submit(_req(0, "a"))
    srv.submit(_req(1, "b"))
    srv.pump()
    # one key set + one request fit; the second client's batch must wait for memory
    assert [l[1] for l in ex.launches] == [[0]]
    clk.t = 1.0
    srv.pump()
    assert [l[1] for l in ex.launches] == [[0], [1]]
    assert srv.evictions == 1


def test_request_that_can_never_fit_is_rejected():
    """With nothing in flight and nothing left to evict, a request whose key set,
    io and workspace exceed the budget is rejected at once (the run ends) while a
    later request that fits is still served."""
    clk = FakeClock()

    class BigKeys(FakeExecutor):
        def key_bytes(self, client, params):
            return 1000 if client == "big" else self.kb

    ex = BigKeys(clk, key_bytes=100, io_per_req=10, ws_per_req=5)
    srv = Server(ex, hbm_budget=300, streams=2, clock=clk)
    for c in ("big", "a"):
        srv.open_session(f"s-{c}", c)
    srv.submit(_req(0, "big"))
    srv.submit(_req(1, "a"))
    srv.pump()
    assert srv.results[0].status == "exceeds the HBM budget"
    assert srv.rejected == 1 and [l[1] for l in ex.launches] == [[1]]
    # through run(): a timeline whose only request never fits ends at once
    import paper_2509_01253_amd.serving as S
    srv2 = Server(BigKeys(clk), hbm_budget=300, streams=2, clock=clk)
    srv2.open_session("s-big", "big")
    orig = S.time.sleep
    S.time.sleep = lambda s: setattr(clk, "t", clk.t + s)
    try:
        res = srv2.run([(0.0, _req(2, "big"))], time_limit=5.0)
    finally:
        S.time.sleep = orig
    assert res[0].status == "exceeds the HBM budget" and srv2.stats(res) == {"completed": 0, "rejected": 1}


def test_run_reports_latency_percentiles():
    clk = FakeClock()

    class TickExecutor(FakeExecutor):
        def done(self, token):
            clk.t += 0.01  # time advances while polling
            return super().done(token)

    ex = TickExecutor(clk, dur=0.05)
    srv = Server(ex, hbm_budget=10 ** 6, streams=2, clock=clk)
    timeline = []
    for i, c in zip(range(20), itertools.cycle("abcd")):
        if i < 4:
            srv.open_session(f"s-{c}", c)
        timeline.append((0.02 * i, _req(i, c, rnd=i // 4 + 1)))
    import paper_2509_01253_amd.serving as S
    orig = S.time.sleep
    S.time.sleep = lambda s: setattr(clk, "t", clk.t + s)
    try:
        res = srv.run(timeline)
    finally:
        S.time.sleep = orig
    st = srv.stats(res)
    assert st["completed"] == 20 and st["rejected"] == 0
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_executor_flags_by_batch_size():
    """A layer registered with (max_batch, flags) pairs runs a batch with the flags of
    the first pair that admits it; the last pair covers every larger batch."""
    from paper_2509_01253_amd.serving import GpuExecutor

    ex = GpuExecutor.__new__(GpuExecutor)  # host logic only: no streams or contexts
    ex.layers = {"a": {"flags": [(1, 3), (4, 1)]}, "b": {"flags": [(1 << 30, 3)]}}
    assert [ex.layer_flags("a", n) for n in (1, 2, 4, 5, 64)] == [3, 1, 1, 1, 1]
    assert [ex.layer_flags("b", n) for n in (1, 64)] == [3, 3]


def test_session_shuffler_permutations():
    """sigma_r depends on the server secret, the session, the round and the unit
    count, is a permutation, is reproducible (the server derives it again for the
    next round's unshuffle), and sigma_0 is the identity."""
    from paper_2509_01253_amd.serving import SessionShuffler
    a = SessionShuffler(b"0123456789abcdef-secret")
    b = SessionShuffler(b"0123456789abcdef-other!")
    p = a.perm("s1", 3, 256)
    assert p.dtype == np.int32 and sorted(p.tolist()) == list(range(256))
    assert np.array_equal(p, a.perm("s1", 3, 256))
    assert a.perm("s1", 0, 256) is None
    others = [a.perm("s2", 3, 256), a.perm("s1", 4, 256), b.perm("s1", 3, 256)]
    assert all(not np.array_equal(p, q) for q in others)
    assert sorted(a.perm("s1", 3, 16).tolist()) == list(range(16))
    with pytest.raises(ValueError):
        SessionShuffler(b"short")
