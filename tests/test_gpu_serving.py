"""Serving loop (continuous batching) on the GPU: streams of different
models, state dimensions and particle counts (up to 2^20) arriving over time
share batched launches in re-bound slots, admitted by their device footprint
against an HBM budget; each stream's result equals the same filter run
alone (states and log-weights bit for bit, estimates to FP32 reduction
order); a stream larger than the budget is rejected and a stream whose
observations turn non-finite fails alone."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _models():
    return {"sv": W.sv_model(), "lg4": W.random_stable_lg(4, 77), "lg16": W.random_stable_lg(16, 78)}


def _requests(models, shapes, n_req=16, rate=300.0, seed=5, T_range=(5, 31)):
    from paper_1812_01502_amd.serving import StreamRequest
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(n_req):
        t += rng.exponential(1.0 / rate)
        name, N = shapes[i % len(shapes)]
        T = int(rng.integers(*T_range))
        _, ys = W.simulate(models[name], T, seed=1000 + i)
        out.append(StreamRequest(stream_id=500 + i, model=name, n_particles=N,
                                 observations=ys.reshape(T, -1), arrival_s=t, seed=9000 + i,
                                 cadence_s=0.002))
    return out


def _check_alone(models, q, res):
    from paper_1812_01502_amd import Filter
    T = q.observations.shape[0]
    m = models[q.model]
    f = Filter(m, q.n_particles, min(64, q.n_particles // 2), seed=q.seed, stream_id=q.stream_id, history=T)
    for y in q.observations:
        f.step(y.astype(np.float32).astype(np.float64))
    xs, ws, ts, lns = f.get_state()
    xb, wb, tb, lnb = res.final_state
    assert ts == tb == T
    assert np.array_equal(xs, xb) and np.array_equal(ws, wb), q.stream_id
    hist = f.history(T)
    for j, h in enumerate(hist):
        sd = np.sqrt(h["var"])
        assert np.all(np.abs(res.means[j] - h["mean"]) <= 1e-5 * np.maximum(np.abs(h["mean"]), sd))
        assert abs(res.log_normaliser[j] - h["log_norm"]) <= 1e-6 * (j + 1)
    assert np.all(np.isfinite(res.latency_s)) and np.all(res.latency_s >= 0)
    f.close()


@pytest.mark.parametrize("realtime", [True, False])
def test_streams_alone_equal_in_mix(realtime):
    from paper_1812_01502_amd.serving import Server, slot_footprint
    models = _models()
    shapes = [("sv", 4096), ("lg4", 2048), ("sv", 1024), ("lg16", 1 << 16), ("sv", 1 << 20), ("lg4", 512)]
    reqs = _requests(models, shapes)
    # room for the 2^20 stream and a little more: admission must wait for
    # memory, not only for slots
    budget = slot_footprint(1, 1 << 20) + slot_footprint(16, 1 << 16) + 4 * slot_footprint(4, 4096)
    log(f"[case] serving {len(reqs)} streams on 6 slots, budget {budget} B, realtime={realtime}")
    srv = Server(models, max_slots=6, hbm_budget=budget, radix=64, pipeline=3, max_substeps=4)
    results, stats = srv.run(reqs, realtime=realtime, keep_final_state=True, max_wall_s=120)
    log(f"   stats {stats}")
    assert stats["streams"] == len(reqs) and stats["rejected_or_failed"] == 0
    assert stats["max_active"] <= 6
    # slots were re-bound: some stream was admitted after another had finished
    fin = min(r.finished_s for r in results.values())
    assert any(r.admitted_s >= fin for r in results.values())
    for q in reqs:
        _check_alone(models, q, results[q.stream_id])
    srv.close()


def test_oversized_rejected_and_nan_stream_fails_alone():
    from paper_1812_01502_amd.serving import Server, StreamRequest, slot_footprint
    models = _models()
    reqs = _requests(models, [("sv", 4096), ("lg4", 2048)], n_req=6, rate=1000.0)
    budget = 8 * slot_footprint(4, 4096)
    big = StreamRequest(stream_id=1, model="sv", n_particles=1 << 22, observations=np.zeros((5, 1)),
                        arrival_s=0.0, seed=3)
    bad_obs = W.simulate(models["lg4"], 12, seed=77)[1]
    bad_obs[6, 2] = np.nan
    bad = StreamRequest(stream_id=2, model="lg4", n_particles=2048, observations=bad_obs, arrival_s=0.001,
                        seed=4, cadence_s=0.002)
    log("[case] serving: oversized stream rejected, NaN stream fails alone")
    srv = Server(models, max_slots=4, hbm_budget=budget, radix=64)
    results, stats = srv.run(reqs + [big, bad], realtime=True, keep_final_state=True, max_wall_s=120)
    log(f"   stats {stats}")
    assert "budget" in results[1].error
    assert "numeric failure at observation 6" in results[2].error
    for q in reqs:
        assert results[q.stream_id].error == ""
        _check_alone(models, q, results[q.stream_id])
    srv.close()
