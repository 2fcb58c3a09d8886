"""Continuous-batching request loop for encrypted linear layers on one GPU.

The server side of the hybrid protocol (paper Sec. 3-4) as a serving system:

* Sessions.  Every request carries a session id and a round counter; a
  request whose round is not the session's next expected round (stale or
  out of order) is rejected (paper Sec. 3, "Clients").
* Clients and keys.  Evaluation keys are uploaded once per client and
  parameter set (paper Sec. 4.2) and stay resident in HBM; under memory
  pressure the least recently used key set with no request in flight is
  evicted (and re-uploaded if the client returns).
* Admission.  A batch is dispatched only if its outputs, input staging,
  workspace growth and missing key sets fit the HBM budget; otherwise the
  requests wait until in-flight work completes and frees memory.  A request
  that does not fit even alone, with nothing in flight and no idle key set
  left to evict, can never run: it is rejected ("exceeds the HBM budget")
  instead of waiting.
* Continuous batching.  Up to `streams` batches are in flight on separate
  HIP streams (two by default: one batch runs while the next is admitted and
  launched; on MI355X four concurrent batches of N=2^16 convolutions ran at
  less than half the throughput of two, each launch already filling the GPU).
  A second batch starts beside a running one only when at least
  `overlap_min_queue` requests wait (two by default).  Whenever a slot frees up, the oldest waiting request and every
  other waiting request for the same layer (any client, any level) form the
  next batch (at most `max_batch` requests), so requests that arrive while
  others run join the next launch and their work overlaps on the device.
* Latency is measured from a request's arrival to the completion of its
  batch; p50 / p99 and throughput are reported.

The GPU work goes through an executor: `GpuExecutor` drives the fhelin C ABI
(one context per parameter set, fhelin_linear_apply_multi for batches mixing
clients); tests substitute a CPU stand-in with the same interface to exercise
the scheduling logic without a GPU.  Results never depend on the batch a
request lands in: every kernel is exact modular arithmetic on per-ciphertext
data.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    client: str
    session: str
    round: int
    layer: str
    level: int
    x: object          # executor-specific input (GPU: tensor [n_in][2][stride][N])
    arrival: float = 0.0  # seconds on the server clock


@dataclass
class Result:
    rid: int
    status: str        # "ok" or the rejection reason
    y: object = None
    level: int = 0
    arrival: float = 0.0
    start: float = 0.0
    end: float = 0.0
    batch: int = 0     # requests in the batch that carried it

    @property
    def latency(self):
        return self.end - self.arrival


@dataclass
class _KeyEntry:
    handle: object
    nbytes: int
    last_used: float
    inflight: int = 0


@dataclass
class _Slot:
    token: object
    reqs: list
    out: object
    nbytes: int
    start: float
    clients: list = field(default_factory=list)


class Server:
    """Request loop; see the module docstring."""

    def __init__(self, executor, hbm_budget: int, streams: int = 2, max_batch: int = 64, clock=time.perf_counter,
                 overlap_min_queue: int = 2):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.n_streams = streams
        self.max_batch = max_batch
        # a batch starts beside one already in flight only when at least this many
        # requests wait: a lone request waits for the running batch instead of
        # sharing the GPU with it (both would run slower, raising the tail latency at
        # light load), while a queue that has built up gets the overlap
        self.overlap_min_queue = overlap_min_queue
        self.clock = clock
        self.sessions = {}                  # session -> next expected round
        self.session_client = {}
        self.keys = collections.OrderedDict()  # (client, params) -> _KeyEntry, LRU order
        self.queue = collections.deque()
        self.inflight = {}                  # stream index -> _Slot
        self.results = {}
        self.live_bytes = 0                 # server-owned tensors (inputs staging, outputs)
        self.rejected = 0
        self.batches = 0
        self.evictions = 0
        self.max_inflight = 0               # most batches on the device at once
        self.batch_s = []                   # dispatch-to-completion time of every batch

    # -- protocol ----------------------------------------------------------
    def open_session(self, session: str, client: str):
        self.sessions[session] = 1
        self.session_client[session] = client

    def submit(self, req: Request) -> bool:
        """Validate (session, round) and enqueue; rejected requests get a Result right away."""
        exp = self.sessions.get(req.session)
        reason = None
        if exp is None:
            reason = "unknown session"
        elif self.session_client.get(req.session) != req.client:
            reason = "session belongs to another client"
        elif req.round != exp:
            reason = f"stale or mismatched round {req.round} (expected {exp})"
        elif not self.ex.has_layer(req.layer):
            reason = f"unknown layer {req.layer}"
        if reason:
            self.rejected += 1
            self.results[req.rid] = Result(req.rid, reason, arrival=req.arrival, start=req.arrival,
                                           end=req.arrival)
            return False
        self.sessions[req.session] = exp + 1
        self.queue.append(req)
        return True

    # -- memory ----------------------------------------------------------
    def used(self) -> int:
        return self.ex.library_bytes() + self.live_bytes

    def _evict_for(self, need: int, protect) -> bool:
        """Evict idle key sets (LRU first) until `need` more bytes fit."""
        while self.used() + need > self.budget:
            victim = next((k for k, e in self.keys.items() if e.inflight == 0 and k not in protect), None)
            if victim is None:
                return False
            e = self.keys.pop(victim)
            self.ex.release_keys(e.handle)
            self.evictions += 1
        return True

    # -- scheduling ------------------------------------------------------
    def _form_batch(self):
        head = self.queue[0]
        batch = [r for r in self.queue if r.layer == head.layer][: self.max_batch]
        return head.layer, batch

    def _try_dispatch(self, stream: int) -> bool:
        if not self.queue:
            return False
        layer, batch = self._form_batch()
        params = self.ex.layer_params(layer)
        need_keys = {(r.client, params) for r in batch if (r.client, params) not in self.keys}
        key_bytes = sum(self.ex.key_bytes(c, p) for c, p in need_keys)
        io_bytes = self.ex.io_bytes(layer, batch)
        ws_bytes = self.ex.workspace_growth(layer, len(batch), stream)
        need = key_bytes + io_bytes + ws_bytes
        protect = {(r.client, params) for r in batch}
        if self.used() + need > self.budget and not self._evict_for(need, protect):
            # shrink the batch until it fits, else wait for completions
            while len(batch) > 1:
                batch = batch[: len(batch) // 2]
                need_keys = {(r.client, params) for r in batch if (r.client, params) not in self.keys}
                need = (sum(self.ex.key_bytes(c, p) for c, p in need_keys) + self.ex.io_bytes(layer, batch)
                        + self.ex.workspace_growth(layer, len(batch), stream))
                protect = {(r.client, params) for r in batch}
                if self.used() + need <= self.budget or self._evict_for(need, protect):
                    break
            else:
                return False
            if self.used() + need > self.budget:
                return False
        now = self.clock()
        handles = []
        for r in batch:
            k = (r.client, params)
            if k not in self.keys:
                h = self.ex.load_keys(r.client, params, stream)
                self.keys[k] = _KeyEntry(h, self.ex.key_bytes(r.client, params), now)
            e = self.keys[k]
            e.inflight += 1
            e.last_used = now
            self.keys.move_to_end(k)
            handles.append(e.handle)
        ids = {id(r) for r in batch}
        self.queue = collections.deque(r for r in self.queue if id(r) not in ids)
        token, out, nbytes = self.ex.launch(layer, batch, handles, stream)
        self.live_bytes += nbytes
        self.inflight[stream] = _Slot(token, batch, out, nbytes, now, [(r.client, params) for r in batch])
        self.batches += 1
        self.max_inflight = max(self.max_inflight, len(self.inflight))
        return True

    def _poll(self) -> int:
        done = 0
        for st, slot in list(self.inflight.items()):
            if not self.ex.done(slot.token):
                continue
            end = self.clock()
            self.batch_s.append(end - slot.start)
            outs = self.ex.collect(slot.token, slot.out, slot.reqs)
            for r, (y, lvl) in zip(slot.reqs, outs):
                self.results[r.rid] = Result(r.rid, "ok", y, lvl, r.arrival, slot.start, end, len(slot.reqs))
            for k in slot.clients:
                if k in self.keys:
                    self.keys[k].inflight -= 1
            self.live_bytes -= slot.nbytes
            del self.inflight[st]
            done += 1
        return done

    def _reject_head(self, reason: str):
        req = self.queue.popleft()
        self.rejected += 1
        now = self.clock()
        self.results[req.rid] = Result(req.rid, reason, arrival=req.arrival, start=now, end=now)

    def pump(self):
        """One scheduling round: retire finished batches, fill free streams."""
        self._poll()
        for st in range(self.n_streams):
            if st not in self.inflight:
                if self.inflight and len(self.queue) < self.overlap_min_queue:
                    break
                while not self._try_dispatch(st):
                    # nothing in flight frees memory later and every idle key set is
                    # already gone: the head request cannot fit, now or later
                    if self.inflight or not self.queue:
                        return
                    self._reject_head("exceeds the HBM budget")
                    if not self.queue:
                        return

    def run(self, timeline, poll_s: float = 2e-4, time_limit: float = 600.0):
        """Serve `timeline`, a list of (arrival_offset_s, Request) sorted by time, in real
        time.  Returns the results in request order."""
        t0 = self.clock()
        i = 0
        while i < len(timeline) or self.queue or self.inflight:
            now = self.clock() - t0
            if now > time_limit:
                raise TimeoutError("serving run exceeded its time limit")
            while i < len(timeline) and timeline[i][0] <= now:
                req = timeline[i][1]
                req.arrival = t0 + timeline[i][0]
                self.submit(req)
                i += 1
            self.pump()
            if not self.inflight and not self.queue and i < len(timeline):
                wait = t0 + timeline[i][0] - self.clock()
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            elif self.inflight:
                time.sleep(poll_s)
        return [self.results[r.rid] for _, r in timeline]

    def stats(self, results) -> dict:
        ok = [r for r in results if r.status == "ok"]
        if not ok:
            return {"completed": 0, "rejected": self.rejected}
        lat = np.array([r.latency for r in ok]) * 1e3
        span = max(r.end for r in ok) - min(r.arrival for r in ok)
        return {
            "completed": len(ok),
            "rejected": self.rejected,
            "throughput_req_s": len(ok) / span if span > 0 else float("inf"),
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_batch": float(np.mean([r.batch for r in ok])),
            "batches": self.batches,
            "max_inflight": self.max_inflight,
            "batch_ms_p50": float(np.percentile(self.batch_s, 50) * 1e3) if self.batch_s else 0.0,
            "batch_ms_max": float(max(self.batch_s) * 1e3) if self.batch_s else 0.0,
            "key_evictions": self.evictions,
        }


class SessionShuffler:
    """The server's secret per-round permutations (paper Sec. 4.4, "Unshuffle" and
    "Shuffle"): sigma_r of a session's round r permutes that round's n output units
    (FC neurons or conv channels) and is drawn from a keyed hash (BLAKE2b keyed with
    the server's secret) of the session id, the round and n, so the server derives it
    again when round r + 1 arrives and needs sigma_r^-1, and the client, who does not
    know the secret, cannot.  sigma_0 = identity (the first layer's input is the
    client's own)."""

    def __init__(self, secret: bytes):
        if len(secret) < 16:
            raise ValueError("the shuffle secret needs at least 16 bytes")
        self.secret = bytes(secret[:64])

    def perm(self, session: str, rnd: int, n: int):
        """sigma_rnd of `session` on n units (int32 array), None for round 0."""
        if rnd <= 0:
            return None
        import hashlib
        h = hashlib.blake2b(f"{session}\x00{int(rnd)}\x00{int(n)}".encode(), key=self.secret, digest_size=16)
        rng = np.random.Generator(np.random.PCG64(int.from_bytes(h.digest(), "little")))
        return rng.permutation(n).astype(np.int32)


def poisson_timeline(rate: float, n: int, stream) -> np.ndarray:
    """Arrival offsets (s) of a Poisson process: cumulative exponential gaps."""
    return np.cumsum(stream.exponential(n, rate))


class GpuExecutor:
    """Executor over the fhelin C ABI (one context per parameter set)."""

    def __init__(self, n_streams: int = 2, flags=None, reserve_requests: int = 0, shuffler=None):
        import torch

        from paper_2509_01253_amd import fhelin as F

        self.torch, self.F = torch, F
        self.flags = (F.FHELIN_APPLY_RESCALE | F.FHELIN_APPLY_HOIST_MODDOWN) if flags is None else flags
        self.params = {}      # name -> dict(ctx, log_n, L, K, ...)
        self.layers = {}      # name -> dict(params, plan, pts, n_in, n_out, ...)
        self.key_src = {}     # (client, params) -> callable(stream) -> (galois, level, evk tensor)
        self.key_size = {}
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.ws = {}          # (params, stream) -> workspace bytes reserved so far
        # > 0: every stream's workspace is grown at registration to a batch of this
        # many requests of each layer, so no batch grows it (a grow synchronises the
        # stream and allocates while requests wait)
        self.reserve_requests = reserve_requests
        # per-round secret permutations of shuffled layers (SessionShuffler)
        self.shuffler = shuffler

    # registration
    def add_params(self, name, log_n, q, p, dnum):
        ctx = self.F.fhelin_ctx_create(log_n, q, p, dnum)
        self.params[name] = dict(ctx=ctx, log_n=log_n, N=1 << log_n, L=len(q), K=len(p), dnum=dnum)

    def add_layer(self, name, params, plan_kwargs, kind, pts, flags=None):
        """flags: this layer's apply flags (its schedule), default the executor's; or a
        list of (max_batch, flags) pairs in increasing max_batch, the last one covering
        every larger batch: a batch runs with the flags of the first pair that admits it.
        With pairs of different schedules a request's output ciphertext depends on the
        size of the batch it ran in (the schedules round differently; both decrypt to
        the layer within the scheme's error); one flags value keeps every output
        bit-identical however the requests are batched."""
        P = self.params[params]
        fl = self.flags if flags is None else flags
        by_batch = [(1 << 30, fl)] if isinstance(fl, int) else [(int(m), int(f)) for m, f in fl]
        by_batch[-1] = (1 << 30, by_batch[-1][1])
        plan = self.F.fhelin_plan_create(P["ctx"], kind, **plan_kwargs)
        info = self.F.fhelin_plan_info(plan)
        self.layers[name] = dict(params=params, plan=plan, pts=pts, n_in=info["n_in"], n_out=info["n_out"],
                                 galois=self.F.fhelin_plan_galois(plan), flags=by_batch)
        if self.reserve_requests > 0:
            # each schedule for the largest batch it runs (at most reserve_requests)
            for i, st in enumerate(self.streams):
                for m, f in by_batch:
                    n = min(self.reserve_requests, m)
                    need = self.F.fhelin_plan_workspace_bytes(P["ctx"], plan, n, f)
                    self.F.fhelin_plan_reserve_workspace(P["ctx"], plan, n, f, stream=st)
                    self.ws[(params, i)] = max(self.ws.get((params, i), 0), need)

    def add_shuffled_layer(self, name, params, plan_kwargs, kind, weights, units_out, units_in, scale,
                           shuffle_out=True, flags=None):
        """A layer whose plaintexts are encoded per request on the GPU with the
        request's session permutations folded in (paper Sec. 4.4): the outputs shuffled
        by sigma_r (unless shuffle_out is False: the network's last layer) and the
        previous round's shuffle undone on the inputs by sigma_{r-1}.  weights: device
        float64 tensor in fhelin_plan_encode_weights' layout; units_out / units_in: the
        lengths of the two permutations (FC neurons or conv channels).  Requests of
        such a layer share no plaintexts: each is encoded at the request's level and
        applied on its own on the batch's stream, and its plaintexts are released when
        the batch completes."""
        if self.shuffler is None:
            raise ValueError("a shuffled layer needs the executor's shuffler")
        self.add_layer(name, params, plan_kwargs, kind, None, flags)
        self.layers[name].update(weights=weights, units_out=int(units_out), units_in=int(units_in),
                                 scale=float(scale), shuffle_out=bool(shuffle_out))

    def request_perms(self, layer, req):
        """(perm_out, perm_in) folded into `req`'s plaintexts (None = identity)."""
        Ly = self.layers[layer]
        po = self.shuffler.perm(req.session, req.round, Ly["units_out"]) if Ly["shuffle_out"] else None
        pi = self.shuffler.perm(req.session, req.round - 1, Ly["units_in"])
        return po, pi

    def _pt_bytes(self, layer, level):
        Ly = self.layers[layer]
        P = self.params[Ly["params"]]
        n_pt = self.F.fhelin_plan_info(Ly["plan"])["n_pt"]
        return n_pt * (level + P["K"]) * P["N"] * 8

    def layer_flags(self, layer, n_req):
        """Apply flags of `layer` for a batch of n_req requests."""
        for m, f in self.layers[layer]["flags"]:
            if n_req <= m:
                return f
        return self.layers[layer]["flags"][-1][1]

    def add_client_keys(self, client, params, source, nbytes):
        """source(stream) -> (galois list, level, evk tensor); nbytes = resident size."""
        self.key_src[(client, params)] = source
        self.key_size[(client, params)] = nbytes

    # executor interface
    def has_layer(self, layer):
        return layer in self.layers

    def layer_params(self, layer):
        return self.layers[layer]["params"]

    def library_bytes(self):
        return sum(self.F.fhelin_ctx_memory(P["ctx"]) for P in self.params.values())

    def key_bytes(self, client, params):
        return self.key_size[(client, params)]

    def io_bytes(self, layer, batch):
        Ly = self.layers[layer]
        P = self.params[Ly["params"]]
        per_ct = 2 * P["L"] * P["N"] * 8
        pts = sum(self._pt_bytes(layer, r.level) for r in batch) if Ly.get("weights") is not None else 0
        return len(batch) * (Ly["n_in"] + Ly["n_out"]) * per_ct + pts

    def workspace_growth(self, layer, n_req, stream):
        Ly = self.layers[layer]
        need = self.F.fhelin_plan_workspace_bytes(self.params[Ly["params"]]["ctx"], Ly["plan"], n_req,
                                                  self.layer_flags(layer, n_req))
        have = self.ws.get((Ly["params"], stream), 0)
        return max(0, need - have)

    def load_keys(self, client, params, stream):
        with self.torch.cuda.stream(self.streams[stream]):
            gal, level, evk = self.key_src[(client, params)](self.streams[stream])
            h = self.F.fhelin_keyset_load(self.params[params]["ctx"], gal, level, evk, stream=self.streams[stream])
        return h

    def release_keys(self, handle):
        self.F.fhelin_keyset_release(handle)

    def launch(self, layer, batch, key_handles, stream):
        torch, F = self.torch, self.F
        Ly = self.layers[layer]
        P = self.params[Ly["params"]]
        s = self.streams[stream]
        L, N = P["L"], P["N"]
        s.wait_stream(torch.cuda.default_stream())  # request inputs were produced on the default stream
        with torch.cuda.stream(s):
            if len(batch) == 1 and batch[0].x.shape[2] == L:
                x = batch[0].x
            else:  # stage the requests into one [R * n_in][2][L][N] batch (inputs may carry only their levels)
                n_in = Ly["n_in"]
                x = torch.empty((len(batch) * n_in, 2, L, N), dtype=torch.int64, device=batch[0].x.device)
                for i, r in enumerate(batch):
                    x[i * n_in:(i + 1) * n_in, :, : r.x.shape[2]] = r.x
            y = torch.empty((len(batch) * Ly["n_out"], 2, L, N), dtype=torch.int64, device=x.device)
            xl = [r.level for r in batch for _ in range(Ly["n_in"])]
            fl = self.layer_flags(layer, len(batch))
            resc = bool(fl & F.FHELIN_APPLY_RESCALE)
            yl = [r.level - (1 if resc else 0) for r in batch for _ in range(Ly["n_out"])]
            own_pts = []
            if Ly.get("weights") is None:
                F.fhelin_linear_apply_multi(P["ctx"], Ly["plan"], key_handles, Ly["pts"], x, xl, y, yl, fl, stream=s)
            else:
                # per-request plaintexts with the request's permutations folded in
                ni, no = Ly["n_in"], Ly["n_out"]
                for i, r in enumerate(batch):
                    po, pi = self.request_perms(layer, r)
                    po = None if po is None else torch.from_numpy(po).to(x.device)
                    pi = None if pi is None else torch.from_numpy(pi).to(x.device)
                    pts = F.fhelin_plan_encode_weights(P["ctx"], Ly["plan"], Ly["weights"], po, pi, r.level,
                                                       Ly["scale"], stream=s)
                    own_pts.append(pts)
                    F.fhelin_linear_apply_multi(P["ctx"], Ly["plan"], key_handles[i:i + 1], pts,
                                                x[i * ni:(i + 1) * ni], xl[i * ni:(i + 1) * ni],
                                                y[i * no:(i + 1) * no], yl[i * no:(i + 1) * no], fl, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        key = (Ly["params"], stream)
        self.ws[key] = max(self.ws.get(key, 0), F.fhelin_plan_workspace_bytes(P["ctx"], Ly["plan"], len(batch), fl))
        return (ev, x, yl, own_pts), y, self.io_bytes(layer, batch)

    def done(self, token):
        return token[0].query()

    def collect(self, token, y, reqs):
        for pts in token[3]:  # per-request plaintexts: the batch has completed
            self.F.fhelin_ptset_release(pts)
        n_out = len(token[2]) // len(reqs)
        return [(y[i * n_out:(i + 1) * n_out], token[2][i * n_out]) for i in range(len(reqs))]

    def close(self):
        self.torch.cuda.synchronize()
        for Ly in self.layers.values():
            self.F.fhelin_plan_destroy(Ly["plan"])
        for P in self.params.values():
            self.F.fhelin_ctx_destroy(P["ctx"])
