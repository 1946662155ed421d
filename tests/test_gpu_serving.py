"""Serving loop (continuous batching) on the GPU: streams arriving over
time share batched launches; each stream's result equals the same filter
run alone (states and log-weights bit for bit, estimates to FP32
reduction order), and slots are reused as streams finish."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _requests(models, n_req=14, rate=300.0, seed=5):
    from paper_1812_01502_amd.serving import StreamRequest
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [("sv", 4096), ("lg4", 2048), ("sv", 1024)]
    t = 0.0
    out = []
    for i in range(n_req):
        t += rng.exponential(1.0 / rate)
        name, N = shapes[int(rng.integers(0, len(shapes)))]
        T = int(rng.integers(5, 31))
        _, ys = W.simulate(models[name], T, seed=1000 + i)
        out.append(StreamRequest(stream_id=500 + i, model=name, n_particles=N,
                                 observations=ys.reshape(T, -1), arrival_s=t, seed=9000 + i,
                                 cadence_s=0.002))
    return out


@pytest.mark.parametrize("realtime", [True, False])
def test_streams_alone_equal_in_mix(realtime):
    from paper_1812_01502_amd import Filter
    from paper_1812_01502_amd.serving import Server
    models = {"sv": W.sv_model(), "lg4": W.random_stable_lg(4, 77)}
    pools = {("sv", 4096): 3, ("lg4", 2048): 2, ("sv", 1024): 2}
    reqs = _requests(models)
    log(f"[case] serving {len(reqs)} streams on {sum(pools.values())} slots, realtime={realtime}")
    srv = Server(models, pools, radix=64)
    results, stats = srv.run(reqs, realtime=realtime, keep_final_state=True, max_wall_s=120)
    log(f"   stats {stats}")
    assert stats["streams"] == len(reqs)
    assert stats["max_concurrent"] <= stats["slots"]
    # slots were reused: some stream was admitted after another had finished
    fin = min(r.finished_s for r in results.values())
    assert any(r.admitted_s >= fin for r in results.values())
    for q in reqs:
        res = results[q.stream_id]
        T = q.observations.shape[0]
        m = models[q.model]
        f = Filter(m, q.n_particles, min(64, q.n_particles // 2), seed=q.seed, stream_id=q.stream_id,
                   history=T)
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
    srv.close()
