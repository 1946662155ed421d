"""Serving loop: continuous batching of filtering streams on one GPU.

A ``Server`` owns one ``BatchFilter`` of ``max_slots`` slots, all vacant at
first, and an HBM budget. Streams arrive over time; each brings its model
(any of the server's models: any state dimension), particle count, seed and
a sequence of observations that become available one by one. The loop

* admits a waiting stream when a slot is free and the stream's device
  footprint fits the unused part of the budget (a stream larger than the
  whole budget is rejected with an error of its own, never raised); the
  admissions and releases of one tick are bound in one ``pf_batch_rebind``
  call (one synchronisation); a finished stream's slot keeps its memory
  until the budget or a new stream needs it,
* on every tick steps every slot that has observations waiting: a slot
  that lags advances through up to ``max_substeps`` of its pending
  observations in the tick, as consecutive batched steps with per-step
  active masks, so streams admitted at different times share the device,
* never waits for the device inside a tick: each tick's observations go to
  the device from page-locked buffers, and its estimate records come back
  with ``pf_batch_estimates_async`` into page-locked buffers behind an event;
  up to ``pipeline`` ticks are in flight, and the host collects a tick's
  estimates when its event has completed,
* records the per-observation latency (estimate in host memory minus the
  time the observation became available) and fails only the stream whose
  record comes back invalid (a numeric failure on the device).

A slot's results depend only on the stream (model, N, radix, seed, stream
id, observations), not on the slot or on the other streams: the batched
kernels compute the same states and log-weights as a single filter.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass

import numpy as np

from . import BatchFilter, ESTIMATE_DTYPE, PfError
from ._lib import PF_E_OOM

__all__ = ["StreamRequest", "StreamResult", "Server", "slot_footprint", "plan_admission"]


@dataclass
class StreamRequest:
    stream_id: int
    model: str                 # key into the server's model table
    n_particles: int
    observations: np.ndarray   # (T, d)
    arrival_s: float = 0.0     # arrival time from the start of the run
    seed: int = 0
    cadence_s: float = 0.0     # observation j is available at arrival + j * cadence


@dataclass
class StreamResult:
    stream_id: int
    slot: int
    admitted_s: float
    finished_s: float = 0.0
    means: np.ndarray = None          # (T, d) filter means, one per observation
    log_normaliser: np.ndarray = None  # (T,)
    latency_s: np.ndarray = None       # (T,) estimate on the host - observation available
    service_s: np.ndarray = None       # (T,) estimate on the host - max(observation available, admission)
    final_state: tuple = None          # (x, logw, t, log_norm) if requested
    error: str = ""                    # why the stream was rejected or failed ("" if served)


CTL_BYTES = 13376    # control block: log-normaliser, offset slots, deferred increments
PARAM_BYTES = 5332   # FP32 model parameters


def slot_footprint(d: int, n: int) -> int:
    """Device bytes of one bound slot: double-buffered states and
    log-weights, tile partial records (each part rounded to 256 bytes as the
    library allocates them), control block, model parameters, record."""
    D = 1 if d <= 1 else 2 if d <= 2 else 4 if d <= 4 else 8 if d <= 8 else 16
    up = lambda v: (v + 63) // 64 * 64  # noqa: E731
    floats = up(2 * d * n) + up(2 * n) + up((n // 512) * (4 + 3 * D))
    return 4 * floats + CTL_BYTES + PARAM_BYTES + 304


def plan_admission(waiting, free, s_shape, s_bytes, budget: int, footprint):
    """Admission of waiting streams in arrival order (first fit).

    ``free``: slots without a stream; ``s_shape[s]``: the (model, N) whose
    memory slot s holds (None: vacant); ``s_bytes[s]``: its bytes;
    ``footprint(r)``: bytes stream r needs (None: unknown model). A stream
    takes a free slot that holds its shape already (no new memory), else a
    vacant one, else the free slot holding the most memory; it is admitted
    if its footprint fits the budget once that slot's memory and, if needed,
    the memory of other free slots (largest first) is given back. Streams
    that can never fit are rejected. Updates ``s_shape`` and ``s_bytes`` and
    returns ``(bind: [(slot, stream)], release: [slot], still waiting:
    [stream], rejected: [(stream, reason)])``."""
    free = list(free)
    used = int(sum(int(v) for v in s_bytes))
    bind, release, still, rejected = [], [], [], []
    for r in waiting:
        fp = footprint(r)
        if fp is None or fp > budget:
            rejected.append((r, "unknown model" if fp is None else
                             f"needs {fp} bytes, more than the HBM budget of {budget}"))
            continue
        if not free:
            still.append(r)
            continue
        shape = (r.model, int(r.n_particles))
        same = [f for f in free if s_shape[f] == shape]
        if same:
            cand = same[0]
        else:
            vac = [f for f in free if s_shape[f] is None]
            held = sorted((f for f in free if s_shape[f] is not None), key=lambda f: -int(s_bytes[f]))
            cand = vac[0] if vac else held.pop(0)
            room = budget - used + int(s_bytes[cand])
            rel = []
            while fp > room and held:
                f = held.pop(0)
                rel.append(f)
                room += int(s_bytes[f])
            if fp > room:
                still.append(r)     # waits for active streams to finish
                continue
            for f in rel:
                used -= int(s_bytes[f])
                s_bytes[f] = 0
                s_shape[f] = None
            release.extend(rel)
            used += fp - int(s_bytes[cand])
        free.remove(cand)
        if cand in release:
            release.remove(cand)
        bind.append((cand, r))
        s_shape[cand] = shape
        s_bytes[cand] = fp
    return bind, release, still, rejected


class _Tick:
    """Buffers of one in-flight tick (page-locked host and device)."""

    def __init__(self, n, y_cap, max_sub):
        import torch
        self.y_host = torch.zeros((max_sub, y_cap), dtype=torch.float32).pin_memory()
        self.a_host = torch.zeros((max_sub, n), dtype=torch.uint8).pin_memory()
        self.y_dev = torch.zeros((max_sub, y_cap), dtype=torch.float32, device="cuda")
        self.a_dev = torch.zeros((max_sub, n), dtype=torch.uint8, device="cuda")
        self.rec_t = torch.empty((max_sub, n * ESTIMATE_DTYPE.itemsize), dtype=torch.uint8).pin_memory()
        self.rec = self.rec_t.numpy().view(ESTIMATE_DTYPE).reshape(max_sub, n)
        self.event = torch.cuda.Event()
        self.steps = []        # per sub-step: (slots, observation indices)
        self.busy = False


class Server:
    """One batch of re-bindable slots and the serving loop over it."""

    def __init__(self, models: dict, max_slots: int = 256, hbm_budget: int = 8 << 30, radix: int = 64,
                 pipeline: int = 3, max_substeps: int = 8):
        """``models``: name -> model (any state dimension); ``max_slots``:
        streams that can be in flight at once; ``hbm_budget``: device bytes
        the slots may hold together."""
        import torch
        self.models = models
        self.radix = radix
        self.n = int(max_slots)
        self.budget = int(hbm_budget)
        self.pipeline = max(1, int(pipeline))
        self.max_sub = max(1, int(max_substeps))
        self.max_d = max(int(m.d) for m in models.values())
        self.stream = torch.cuda.Stream()
        self.batch = BatchFilter([None] * self.n, [0] * self.n, [0] * self.n, [0] * self.n,
                                 stream=self.stream.cuda_stream)

    def close(self):
        self.batch.close()

    def footprint(self, r: StreamRequest) -> int:
        return slot_footprint(int(self.models[r.model].d), int(r.n_particles))

    def run(self, requests, realtime: bool = True, keep_final_state: bool = False,
            max_wall_s: float = 600.0):
        """Serve ``requests`` to completion. ``realtime``: arrivals and
        observation times follow the wall clock; otherwise every stream has
        arrived with all its observations available (saturation). Returns
        ``(results by stream_id, stats)``."""
        import torch
        b = self.batch
        n = self.n
        requests = sorted(requests, key=lambda r: r.arrival_s)
        ticks = [_Tick(n, n * self.max_d, self.max_sub) for _ in range(self.pipeline)]
        inflight = collections.deque()
        # per-slot state
        s_req = [None] * n            # stream bound to the slot (None: free)
        s_shape = [None] * n          # (model, N) the slot's memory holds (None: vacant)
        s_bytes = np.zeros(n, dtype=np.int64)
        s_arr = np.zeros(n)
        s_cad = np.zeros(n)
        s_T = np.zeros(n, dtype=np.int64)
        s_sub = np.zeros(n, dtype=np.int64)     # observations submitted
        s_done = np.zeros(n, dtype=np.int64)    # estimates collected
        s_adm = np.zeros(n)
        s_obs = [None] * n
        s_out = [None] * n                      # (means, log-norm, latency, service)
        pending = collections.deque(requests)
        waiting = collections.deque()
        results = {}
        counters = dict(ticks=0, substeps=0, stream_steps=0, particle_steps=0, rebinds=0, max_active=0)
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        def finish(s, now, error=""):
            r = s_req[s]
            T = int(s_T[s])
            means, ln, lat, svc = s_out[s]
            res = StreamResult(r.stream_id, int(s), admitted_s=float(s_adm[s]), finished_s=now,
                               means=means, log_normaliser=ln, latency_s=lat, service_s=svc, error=error)
            if keep_final_state and not error:
                res.final_state = b.get_state(int(s))
            results[r.stream_id] = res
            if not error:
                counters["particle_steps"] += T * int(r.n_particles)
            s_req[s] = None

        def collect(tk, now):
            """Estimates of a completed tick into the streams' buffers."""
            for k, (slots, idx) in enumerate(tk.steps):
                rec = tk.rec[k, slots]
                for s, j, rr in zip(slots.tolist(), idx.tolist(), rec):
                    if s_req[s] is None:
                        continue           # failed earlier in this tick
                    means, ln, lat, svc = s_out[s]
                    d = means.shape[1]
                    means[j] = rr["mean"][:d]
                    ln[j] = rr["log_normaliser"]
                    avail = s_arr[s] + j * s_cad[s]
                    lat[j] = now - avail if realtime else 0.0
                    svc[j] = now - max(avail, s_adm[s]) if realtime else 0.0
                    s_done[s] = max(s_done[s], j + 1)
                    if rr["valid"] != 1:
                        finish(s, now, error=f"numeric failure at observation {j}")
                    elif s_done[s] >= s_T[s]:
                        finish(s, now)
            tk.steps = []
            tk.busy = False

        def admit(now):
            while pending and (not realtime or pending[0].arrival_s <= now):
                waiting.append(pending.popleft())
            if not waiting:
                return
            free = [s for s in range(n) if s_req[s] is None]
            bind, release, still, rejected = plan_admission(
                waiting, free, s_shape, s_bytes, self.budget,
                lambda r: self.footprint(r) if r.model in self.models else None)
            waiting.clear()
            for r, why in rejected:
                results[r.stream_id] = StreamResult(r.stream_id, -1, admitted_s=now, finished_s=now, error=why)
            waiting.extend(still)
            if not bind and not release:
                return
            # in-flight ticks complete before the slots change
            while inflight:
                tk = inflight.popleft()
                tk.event.synchronize()
                collect(tk, clock())
            try:
                b.rebind([(f, None, 0, 0, 0, 0) for f in release] +
                         [(s, self.models[r.model], r.n_particles, min(self.radix, r.n_particles // 2),
                           r.seed, r.stream_id) for s, r in bind])
            except PfError as e:
                if e.status != PF_E_OOM:
                    raise
                # the device had less memory than the budget: streams whose
                # slot stayed vacant wait again
                for s, r in list(bind):
                    if b.ns[s] == 0:
                        bind.remove((s, r))
                        s_shape[s] = None
                        s_bytes[s] = 0
                        waiting.appendleft(r)
            counters["rebinds"] += 1
            now = clock()
            for s, r in bind:
                d = int(self.models[r.model].d)
                obs = np.asarray(r.observations, dtype=np.float32).reshape(-1, d)
                T = obs.shape[0]
                s_req[s] = r
                s_obs[s] = obs
                s_arr[s] = r.arrival_s if realtime else 0.0
                s_cad[s] = r.cadence_s if realtime else 0.0
                s_T[s] = T
                s_sub[s] = 0
                s_done[s] = 0
                s_adm[s] = now
                s_out[s] = (np.zeros((T, d)), np.zeros(T), np.zeros(T), np.zeros(T))
            counters["max_active"] = max(counters["max_active"], sum(x is not None for x in s_req))

        def submit(now):
            """One tick of up to max_substeps batched steps; False if idle."""
            act = np.array([s for s in range(n) if s_req[s] is not None and s_sub[s] < s_T[s]], dtype=np.int64)
            if act.size == 0:
                return False
            if realtime:
                avail = np.floor((now - s_arr[act]) / np.maximum(s_cad[act], 1e-12)).astype(np.int64) + 1
                avail = np.where(s_cad[act] > 0, avail, s_T[act])
            else:
                avail = s_T[act]
            backlog = np.minimum(np.minimum(avail, s_T[act]) - s_sub[act], self.max_sub)
            K = int(backlog.max()) if backlog.size else 0
            if K <= 0:
                return False
            if len(inflight) == self.pipeline:
                tk = inflight.popleft()
                tk.event.synchronize()
                collect(tk, clock())
            tk = next(t for t in ticks if not t.busy)
            offs = b.y_offsets
            yh, ah = tk.y_host.numpy(), tk.a_host.numpy()
            with torch.cuda.stream(self.stream):
                for k in range(K):
                    sel = act[backlog > k]
                    idx = s_sub[sel] + k
                    ah[k, :] = 0
                    ah[k, sel] = 1
                    for s, j in zip(sel.tolist(), idx.tolist()):
                        o = int(offs[s])
                        yh[k, o:o + s_obs[s].shape[1]] = s_obs[s][j]
                    tk.y_dev[k].copy_(tk.y_host[k], non_blocking=True)
                    tk.a_dev[k].copy_(tk.a_host[k], non_blocking=True)
                    b.step(tk.y_dev[k].data_ptr(), tk.a_dev[k].data_ptr())
                    b.estimates_async(tk.rec[k])
                    tk.steps.append((sel, idx))
                    counters["stream_steps"] += int(sel.size)
                tk.event.record(self.stream)
            s_sub[act] += backlog
            tk.busy = True
            inflight.append(tk)
            counters["ticks"] += 1
            counters["substeps"] += K
            return True

        while pending or waiting or any(x is not None for x in s_req):
            now = clock()
            if now > max_wall_s:
                raise TimeoutError("serving run exceeded its wall-clock limit")
            while inflight and inflight[0].event.query():
                collect(inflight.popleft(), clock())
            admit(now)
            if not submit(clock()):
                if inflight:
                    tk = inflight.popleft()
                    tk.event.synchronize()
                    collect(tk, clock())
                else:
                    nxt = [pending[0].arrival_s] if pending else []
                    nxt += [s_arr[s] + s_sub[s] * s_cad[s] for s in range(n)
                            if s_req[s] is not None and s_sub[s] < s_T[s]]
                    if nxt:
                        wait = min(nxt) - clock()
                        if wait > 0:
                            time.sleep(min(wait, 0.0005))
        wall = clock()
        served = [r for r in results.values() if not r.error]
        lat = np.concatenate([r.latency_s for r in served]) if served else np.zeros(1)
        svc = np.concatenate([r.service_s for r in served]) if served else np.zeros(1)
        by_id = {q.stream_id: q for q in requests}
        wait = np.array([r.admitted_s - by_id[r.stream_id].arrival_s for r in served]) if (served and realtime) \
            else np.zeros(1)
        stats = dict(wall_s=wall, particle_steps_per_s=counters["particle_steps"] / wall,
                     streams=len(served), rejected_or_failed=len(results) - len(served),
                     slots=n, hbm_budget=self.budget,
                     latency_p50_ms=float(np.percentile(lat, 50) * 1e3),
                     latency_p99_ms=float(np.percentile(lat, 99) * 1e3),
                     service_latency_p50_ms=float(np.percentile(svc, 50) * 1e3),
                     service_latency_p99_ms=float(np.percentile(svc, 99) * 1e3),
                     admission_wait_p50_ms=float(np.percentile(wait, 50) * 1e3),
                     admission_wait_p99_ms=float(np.percentile(wait, 99) * 1e3), **counters)
        return results, stats
