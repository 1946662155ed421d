"""Serving loop: continuous batching of filtering streams on one GPU.

A ``Server`` owns pools of filter slots, one pool per (model, N) shape, all
in one ``BatchFilter`` (one launch per dimension class and step). Streams
arrive over time; each brings its model, particle count, seed and a
sequence of observations that become available one by one. The loop

* admits a waiting stream as soon as a slot of its shape is free (slots are
  sized up front from an HBM budget by their device footprint) and
  re-initialises that slot with the stream's seed and stream id,
* on every tick steps all slots that have an observation waiting, in one
  batched launch, so streams admitted at different times share the device,
* reads the estimate of every stepped slot, records the per-observation
  latency (estimate on the host minus the time the observation became
  available), and frees the slot when its stream has no observations left.

A slot's results depend only on the stream (model, N, radix, seed, stream
id, observations), not on the slot or on the other streams: the batched
kernels guarantee the same states and log-weights as a single filter.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import BatchFilter, ESTIMATE_DTYPE

__all__ = ["StreamRequest", "StreamResult", "Server", "slot_footprint", "slots_for_budget"]


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
    latency_s: np.ndarray = None       # (T,) estimate ready - observation available
    service_s: np.ndarray = None       # (T,) estimate ready - max(observation available, admission)
    final_state: tuple = None          # (x, logw, t, log_norm) if requested


CTL_BYTES = 13376    # control block: log-normaliser, offset slots, deferred increments
PARAM_BYTES = 5332   # FP32 model parameters


def slot_footprint(d: int, n: int) -> int:
    """Device bytes of one slot: double-buffered states and log-weights,
    tile partial records, control block, model parameters, record."""
    D = 1 if d <= 1 else 2 if d <= 2 else 4 if d <= 4 else 8 if d <= 8 else 16
    return 2 * d * n * 4 + 2 * n * 4 + (n // 512) * (4 + 3 * D) * 4 + CTL_BYTES + PARAM_BYTES + 304


def slots_for_budget(shapes: dict, dims: dict, hbm_budget: int) -> dict:
    """Slot counts per shape ``(model, N)`` from relative demand weights
    ``shapes[(model, N)]`` so that the pools fit ``hbm_budget`` bytes."""
    tot_w = float(sum(shapes.values()))
    out = {}
    for (m, n), w in shapes.items():
        share = hbm_budget * (w / tot_w)
        out[(m, n)] = max(1, int(share // slot_footprint(dims[m], n)))
    return out


class Server:
    """Pools of batched filter slots and the serving loop over them."""

    def __init__(self, models: dict, pools: dict, radix: int = 64, stream: int | None = None):
        """``models``: name -> model; ``pools``: (name, N) -> number of slots."""
        self.models = models
        self.radix = radix
        self.shape_of_slot = []
        for (name, n), cnt in sorted(pools.items()):
            self.shape_of_slot += [(name, int(n))] * int(cnt)
        ms = [models[nm] for nm, _ in self.shape_of_slot]
        ns = [n for _, n in self.shape_of_slot]
        self.batch = BatchFilter(ms, ns, [min(radix, n // 2) for n in ns],
                                 seeds=list(range(len(ms))), stream=stream)
        self.n = len(ms)
        self.ds = np.array([m.d for m in ms])
        self.free = collections.defaultdict(collections.deque)
        for s, shape in enumerate(self.shape_of_slot):
            self.free[shape].append(s)
        self.device_bytes = sum(slot_footprint(m.d, n) for m, n in zip(ms, ns))

    def close(self):
        self.batch.close()

    def run(self, requests, realtime: bool = True, keep_final_state: bool = False,
            max_wall_s: float = 600.0):
        """Serve ``requests`` to completion. ``realtime``: arrivals and
        observation times are honoured against the wall clock; otherwise
        every stream is treated as arrived with all observations available
        (saturation). Returns ``(results by stream_id, stats)``."""
        import torch
        b = self.batch
        n = self.n
        requests = list(requests)
        T_max = max(int(r.observations.shape[0]) for r in requests)
        y_host = torch.zeros(b.y_len, dtype=torch.float32).pin_memory()
        a_host = torch.zeros(n, dtype=torch.uint8).pin_memory()
        y_dev = torch.zeros(b.y_len, dtype=torch.float32, device="cuda")
        a_dev = torch.zeros(n, dtype=torch.uint8, device="cuda")
        yh, ah = y_host.numpy(), a_host.numpy()
        rec = np.empty(n, dtype=ESTIMATE_DTYPE)
        offs = np.asarray(b.y_offsets)
        # per-slot state of the loop, as arrays
        s_req = [None] * n
        s_act = np.zeros(n, dtype=bool)
        s_arr = np.zeros(n)
        s_cad = np.zeros(n)
        s_T = np.zeros(n, dtype=np.int64)
        obs_idx = np.zeros(n, dtype=np.int64)
        lat_buf = np.zeros((n, T_max))
        svc_buf = np.zeros((n, T_max))
        ln_buf = np.zeros((n, T_max))
        adm = np.zeros(n)
        groups = {}
        for d in sorted(set(self.ds.tolist())):
            slots = np.nonzero(self.ds == d)[0]
            row = np.full(n, -1, dtype=np.int64)
            row[slots] = np.arange(slots.size)
            groups[d] = (slots, row, np.zeros((slots.size, T_max, d), dtype=np.float32),
                         np.zeros((slots.size, T_max, d)), np.arange(d))
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        waiting = collections.deque()
        results = {}
        stream_steps = 0
        particle_steps = 0
        ticks = 0
        max_active = 0
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        def admit(now):
            nonlocal max_active
            while pending and (not realtime or pending[0].arrival_s <= now):
                waiting.append(pending.popleft())
            still = collections.deque()
            while waiting:
                r = waiting.popleft()
                shape = (r.model, int(r.n_particles))
                if shape not in self.free:
                    raise ValueError(f"no pool serves {shape}")
                if not self.free[shape]:
                    still.append(r)
                    continue
                s = self.free[shape].popleft()
                b.reset(s, seed=r.seed, stream_id=r.stream_id)
                d = int(self.ds[s])
                obs = np.asarray(r.observations, dtype=np.float32).reshape(-1, d)
                slots, row, buf, _, _ = groups[d]
                buf[row[s], :obs.shape[0]] = obs
                s_req[s] = r
                s_act[s] = True
                s_arr[s] = r.arrival_s if realtime else 0.0
                s_cad[s] = r.cadence_s if realtime else 0.0
                s_T[s] = obs.shape[0]
                obs_idx[s] = 0
                adm[s] = clock()
            waiting.extend(still)
            max_active = max(max_active, int(s_act.sum()))

        while pending or waiting or s_act.any():
            if clock() > max_wall_s:
                raise TimeoutError("serving run exceeded its wall-clock limit")
            now = clock()
            admit(now)
            avail = s_arr + obs_idx * s_cad
            ready = s_act & (avail <= now) if realtime else s_act.copy()
            act = np.nonzero(ready)[0]
            if act.size == 0:
                nxt = []
                if pending:
                    nxt.append(pending[0].arrival_s)
                if s_act.any():
                    nxt.append(float(np.min(avail[s_act])))
                if nxt:
                    wait = min(nxt) - clock()
                    if wait > 0:
                        time.sleep(min(wait, 0.001))
                continue
            for d, (slots, row, buf, _, ar) in groups.items():
                sel = act[self.ds[act] == d]
                if sel.size:
                    yh[(offs[sel][:, None] + ar[None, :]).ravel()] = buf[row[sel], obs_idx[sel]].ravel()
            ah[:] = 0
            ah[act] = 1
            y_dev.copy_(y_host, non_blocking=True)
            a_dev.copy_(a_host, non_blocking=True)
            torch.cuda.current_stream().synchronize()
            b.step(y_dev.data_ptr(), a_dev.data_ptr())
            b.estimates_array(rec)
            done = clock()
            ticks += 1
            j = obs_idx[act]
            for d, (slots, row, _, means, _) in groups.items():
                sel = act[self.ds[act] == d]
                if sel.size:
                    means[row[sel], obs_idx[sel]] = rec["mean"][sel, :d]
            ln_buf[act, j] = rec["log_normaliser"][act]
            lat_buf[act, j] = (done - avail[act]) if realtime else 0.0
            svc_buf[act, j] = (done - np.maximum(avail[act], adm[act])) if realtime else 0.0
            obs_idx[act] = j + 1
            stream_steps += int(act.size)
            for s in act[obs_idx[act] >= s_T[act]]:
                r = s_req[s]
                T = int(s_T[s])
                d = int(self.ds[s])
                _, row, _, means, _ = groups[d]
                res = StreamResult(r.stream_id, int(s), admitted_s=float(adm[s]), finished_s=done,
                                   means=means[row[s], :T].copy(), log_normaliser=ln_buf[s, :T].copy(),
                                   latency_s=lat_buf[s, :T].copy(), service_s=svc_buf[s, :T].copy())
                if keep_final_state:
                    res.final_state = b.get_state(int(s))
                results[r.stream_id] = res
                particle_steps += T * int(r.n_particles)
                s_req[s] = None
                s_act[s] = False
                self.free[(r.model, int(r.n_particles))].append(int(s))
        wall = clock()
        lat = np.concatenate([r.latency_s for r in results.values()]) if results else np.zeros(1)
        svc = np.concatenate([r.service_s for r in results.values()]) if results else np.zeros(1)
        wait = np.array([r.admitted_s - q.arrival_s for q in requests
                         for r in [results.get(q.stream_id)] if r is not None]) if realtime else np.zeros(1)
        stats = dict(wall_s=wall, ticks=ticks, stream_steps=stream_steps, particle_steps=particle_steps,
                     particle_steps_per_s=particle_steps / wall, streams=len(results),
                     max_concurrent=max_active, slots=n, device_bytes=self.device_bytes,
                     latency_p50_ms=float(np.percentile(lat, 50) * 1e3),
                     latency_p99_ms=float(np.percentile(lat, 99) * 1e3),
                     service_latency_p50_ms=float(np.percentile(svc, 50) * 1e3),
                     service_latency_p99_ms=float(np.percentile(svc, 99) * 1e3),
                     admission_wait_p50_ms=float(np.percentile(wait, 50) * 1e3),
                     admission_wait_p99_ms=float(np.percentile(wait, 99) * 1e3))
        return results, stats
