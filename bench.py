"""Benchmark of the butterfly-interaction particle filter on one MI355X.

Workload (default): the 8-D linear-Gaussian model (A = 0.9 I + 0.05 O, Q = I,
H = I, R = 0.5 I), N = 2^20 particles, radix 64 (stages 64, 64, 64, 4),
multinomial resampling, FP32 states and log-weights, FP64 log-normaliser;
synthetic observations simulated from the model (seed 2). One "step" is one
filter time step over all N particles: log-weight -> group resample ->
gather -> propagate (+ estimate partials and the final reduction).

Printed (one JSON line): particle-steps/s of the butterfly path with the
observations already in device memory, the global-resampling bootstrap
filter (r = N) on the same input and its speedup, p50/p99 step latency,
the roofline of the step kernel (algorithmic bytes / measured time against
the 8 TB/s HBM peak), and the FP64 oracle timed on the host as a baseline.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--radix 64]
       python bench.py --mode profile   (kernel-only run for rocprofv3)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# rocprofv3 counter summaries of the step kernel, per workload
PROFILE_SUMMARY = {"lg8": os.path.join(ROOT, "profiles", "pf_step_tile_lg8_n2p20_r64.json"),
                   "sv": os.path.join(ROOT, "profiles", "pf_step_tile_sv_n2p24_r64.json")}
KERNEL_SOURCES = ["paper_1812_01502_amd/csrc/pf_kernels.h", "paper_1812_01502_amd/csrc/pf_device.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(d: int, state_bytes: int, path: str) -> int:
    """Bytes one particle-step must move. Butterfly (fused): read and write
    x (d components) and the FP32 log-weight once. Global bootstrap filter:
    the cheaper of re-reading x (4 d s) or storing a CDF and ancestor
    (2 d s + 16); log-weights are all zero after a global resample."""
    if path == "butterfly":
        return 2 * (d * state_bytes + 4)
    return min(4 * d * state_bytes, 2 * d * state_bytes + 16)


def timed_run(flt, yd, steps, d):
    import torch
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    flt.run(yd.data_ptr(), steps, d)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, start.elapsed_time(stop) / 1e3


def per_step_latency(flt, yd, steps, d):
    import numpy as np
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    for j in range(steps):
        evs[j][0].record()
        flt.run(yd[j].data_ptr(), 1, d)
        evs[j][1].record()
    torch.cuda.synchronize()
    us = np.array([a.elapsed_time(b) * 1e3 for a, b in evs])
    return float(np.percentile(us, 50)), float(np.percentile(us, 99)), float(us.mean())


def cpu_baseline(model, N, radix, ys, budget_s=12.0):
    """The FP64 oracle as it stands, single-threaded, on the same workload:
    as many time steps of N particles as fit in about budget_s seconds."""
    from threadpoolctl import threadpool_limits
    from oracle import ButterflyOracle
    with threadpool_limits(limits=1):
        orc = ButterflyOracle(model, N, radix, seed=202)
        st = orc.init()
        t0 = time.perf_counter()
        n = 0
        while n < len(ys):
            st, _ = orc.step(st, ys[n], keep=False)
            n += 1
            if time.perf_counter() - t0 > budget_s:
                break
        el = time.perf_counter() - t0
    return dict(value=N * n / el, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"{n} time steps of N = {N} particles, radix {radix} "
                       f"(stage cycle {orc.plan}), FP64 NumPy, 1 thread, {el:.1f} s")


def batched_bench(steps: int, warmup: int):
    """The batched workload: 4096 independent LG filters, N_f = 2^u with u
    uniform in 10..16, d_f uniform over {1, 4, 16}, seeded stable A, radix and
    tile chosen by the autotuner; the timed steps run as one HIP graph."""
    import numpy as np
    import torch
    import paper_1812_01502_amd as P
    import workloads as W
    t0 = time.perf_counter()
    models, Ns, Y = W.batched_workload(T=warmup + steps)
    gen_s = time.perf_counter() - t0
    ds = [m.d for m in models]
    yd = torch.tensor(Y, dtype=torch.float32, device="cuda").contiguous()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    t0 = time.perf_counter()
    b = P.BatchFilter(models, Ns, [0] * len(models), [404 + f for f in range(len(models))],
                      stream=s.cuda_stream)
    create_s = time.perf_counter() - t0
    with torch.cuda.stream(s):
        b.run(yd.data_ptr(), warmup)
        b.sync()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(s)
        b.run(yd[warmup:].data_ptr(), steps, use_graph=True)
        ev1.record(s)
        b.sync()
        wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    recs = b.estimates()
    tune = b.tuning()
    b.close()
    n_part = int(sum(Ns))
    bytes_step = int(sum(N * (2 * (d * 4 + 4)) for N, d in zip(Ns, ds)))
    chosen = sorted({(t["dim"], t["radix"], t["ppt"]) for t in tune if t["chosen"]})
    return {
        "workload": "4096 LG filters, N in 2^10..2^16, d in {1, 4, 16}, autotuned radix/tile",
        "filters": len(models), "particles": n_part, "steps": steps,
        "particle_steps_per_s": n_part * steps / wall,
        "ms_per_step": wall / steps * 1e3,
        "graph_gpu_ms_per_step": gpu_s / steps * 1e3,
        "hbm_frac_algorithmic": bytes_step / (gpu_s / steps) / 1e9 / HBM_PEAK_GBS,
        "bytes_per_step": bytes_step,
        "autotuned": [{"dim": d, "radix": r, "tile": 512 * p} for d, r, p in chosen],
        "create_s": create_s, "input_generation_s": gen_s,
        "all_valid": bool(all(r["valid"] for r in recs)),
    }


def serving_bench(window_s: float = 1.0, rate: float = 2000.0, seed: int = 5):
    """The serving workload: Poisson arrivals (``rate`` streams/s over
    ``window_s``) of SV or 4-D LG streams (half each), N uniform over
    {2^12, 2^16, 2^20}, 50..500 observations each, one observation per
    millisecond; slot pools sized from the expected concurrency within an
    HBM budget; continuous batching on one GPU."""
    import math
    import numpy as np
    import workloads as W
    from paper_1812_01502_amd.serving import Server, StreamRequest, slot_footprint
    rng = np.random.Generator(np.random.PCG64(seed))
    models = {"sv": W.sv_model(), "lg4": W.random_stable_lg(4, 5004)}
    Ns = [1 << 12, 1 << 16, 1 << 20]
    cadence = 1e-3
    t, reqs = 0.0, []
    sim = {}
    while True:
        t += rng.exponential(1.0 / rate)
        if t > window_s:
            break
        name = "sv" if rng.random() < 0.5 else "lg4"
        N = Ns[int(rng.integers(0, 3))]
        T = int(rng.integers(50, 501))
        if name not in sim:   # one long simulated path per model; streams take windows of it
            sim[name] = W.simulate(models[name], 20000, seed=seed)[1].reshape(20000, -1)
        o = int(rng.integers(0, 20000 - T))
        reqs.append(StreamRequest(stream_id=len(reqs), model=name, n_particles=N,
                                  observations=sim[name][o:o + T], arrival_s=t,
                                  seed=77 + len(reqs), cadence_s=cadence))
    budget = 24 << 30
    mean_T = 275.0
    pools = {}
    for name in models:
        for N in Ns:
            want = math.ceil(1.5 * rate / 6.0 * mean_T * cadence)
            cap = int((budget / 6) // slot_footprint(models[name].d, N))
            pools[(name, N)] = max(1, min(want, cap))
    srv = Server(models, pools, radix=64)
    _, stats = srv.run(reqs, realtime=True, max_wall_s=300)
    srv.close()
    stats.update(workload=f"Poisson {rate:g}/s over {window_s:g} s, SV or LG-4, N in 2^12/2^16/2^20, "
                          f"50..500 observations at 1 ms", pools={f"{k[0]} N={k[1]}": v for k, v in pools.items()})
    return stats


def island_size(args, N: int) -> int:
    """Island size of the island-filter section: 1024 particles (LG-8,
    2^20 particles: 1024 islands), 4096 (SV, 2^24: 4096 islands)."""
    if args.island:
        return args.island
    return min(1024 if args.workload == "lg8" else 4096, N // 2)


def island_bytes(d: int, state_bytes: int) -> int:
    """Bytes one island-filter particle-step must move with its three
    launches: the within-island launch reads x and writes the ancestor
    (the incoming log-weights are all zero and not read); the gather reads
    the ancestor and x and writes x."""
    return 3 * d * state_bytes + 8


def adaptive_bytes(d: int, state_bytes: int, stages: float) -> float:
    """Bytes one particle-step with ESS-gated stages must move: the
    weighting reads x and the log-weight and writes the log-weight; every
    stage run reads and writes both in place; the mutation reads both and
    writes both to the other buffers."""
    row = d * state_bytes + 4
    return (row + 4) + 2 * row * stages + 2 * row


def load_traffic(path, n_launch_bytes):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel sources; else None."""
    try:
        with open(path) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    if prof.get("kernel_source_hash") != kernel_source_hash():
        return None
    return prof.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=500,
                    help="untimed steps first: the step time settles after a few hundred launches")
    ap.add_argument("--radix", type=int, default=64)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--mode", choices=["bench", "profile"], default="bench")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extra-radices", default="2,4,32")
    ap.add_argument("--workload", choices=["lg8", "sv"], default="lg8",
                    help="lg8: 8-D LG, N = 2^20 (default); sv: stochastic volatility, N = 2^24")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-filters section")
    ap.add_argument("--batch-only", action="store_true", help="print only the batched-filters section")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--serve-only", action="store_true", help="print only the serving section")
    ap.add_argument("--island", type=int, default=0, help="island size of the island-filter section")
    ap.add_argument("--profile-island", action="store_true",
                    help="--mode profile: run the island filter instead of the butterfly filter")
    ap.add_argument("--profile-adaptive", action="store_true",
                    help="--mode profile: run the ESS-gated filter (theta 0.5) instead")
    ap.add_argument("--serve-window", type=float, default=1.0, help="arrival window of the serving run (s)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1812_01502_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    P.load_library()
    if args.batch_only:
        print(json.dumps({"batched": batched_bench(200, 5)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serving_bench(args.serve_window)}), flush=True)
        return
    cfg = W.config("c2" if args.workload == "lg8" else "c3")
    if args.workload == "sv" and args.n == 1 << 20:
        args.n = cfg["N"]
    model, N, d = cfg["model"], args.n, cfg["model"].d
    K, Wm = args.steps, args.warmup
    _, ys = W.simulate(model, Wm + K, seed=cfg["seed_obs"])
    yd = torch.tensor(ys, dtype=torch.float32, device="cuda").contiguous()
    stream = torch.cuda.current_stream()

    def make(radix, full_cycle=False):
        return P.Filter(model, N, radix, seed=cfg["seed_pf"], history=4,
                        stream=stream.cuda_stream, full_cycle=full_cycle)

    def make_island(M):
        return P.Filter(model, N, 2, seed=cfg["seed_pf"], history=4, stream=stream.cuda_stream, island=M)

    if args.mode == "profile":
        # step kernels only (for rocprofv3), then a plain copy of known size
        if args.profile_island:
            flt = make_island(island_size(args, N))
        elif args.profile_adaptive:
            flt = P.Filter(model, N, args.radix, seed=cfg["seed_pf"], history=4, stream=stream.cuda_stream,
                           ess_threshold=0.5)
        else:
            flt = make(args.radix)
        flt.run(yd.data_ptr(), Wm, d)
        wall, ev_s = timed_run(flt, yd[Wm:], K, d)
        flt.close()
        src = torch.empty(1 << 27, dtype=torch.float32, device="cuda")   # 512 MiB
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "copy_bytes": src.numel() * 4, "warmup": Wm, "steps": K,
                          "avg_launch_us": ev_s / K * 1e6}))
        return

    # -- butterfly, headline radix ------------------------------------------
    flt = make(args.radix)
    plan = flt.info()["stages"]
    flt.run(yd.data_ptr(), Wm, d)                     # warm-up steps
    wall, ev_s = timed_run(flt, yd[Wm:], K, d)
    value = N * K / wall
    ms_step = wall / K * 1e3
    p50, p99, mean_us = per_step_latency(flt, yd, min(K, Wm + K), d)
    est = flt.estimate()
    flt.close()
    B = algorithmic_bytes(d, 4, "butterfly")
    launch_bytes = B * N
    avg_launch_s = ev_s / K                            # one step kernel per step
    achieved = launch_bytes / avg_launch_s / 1e9
    # the counters were taken at the workload's own N only
    traffic = load_traffic(PROFILE_SUMMARY[args.workload], launch_bytes) if N == cfg["N"] else None

    # -- global bootstrap filter (r = N) ---------------------------------------
    g = make(N)
    g.run(yd.data_ptr(), Wm, d)
    gwall, gev = timed_run(g, yd[Wm:], K, d)
    gvalue = N * K / gwall
    gp50, gp99, _ = per_step_latency(g, yd, min(K, Wm + K), d)
    g.close()
    Bg = algorithmic_bytes(d, 4, "global")

    # -- other radices --------------------------------------------------------
    per_radix = {}
    for r in [int(v) for v in args.extra_radices.split(",") if v]:
        f2 = make(r)
        f2.run(yd.data_ptr(), Wm, d)
        w2, e2 = timed_run(f2, yd[Wm:], K, d)
        per_radix[str(r)] = dict(particle_steps_per_s=N * K / w2, ms_per_step=w2 / K * 1e3,
                                 hbm_frac=B * N / (e2 / K) / 1e9 / HBM_PEAK_GBS,
                                 stages=f2.info()["stages"])
        f2.close()
    per_radix[str(args.radix)] = dict(particle_steps_per_s=value, ms_per_step=ms_step,
                                      hbm_frac=achieved / HBM_PEAK_GBS, stages=plan)

    # -- full augmented resampling per step (all S stages, Algorithm 3) ----------
    fc = make(args.radix, full_cycle=True)
    fc.run(yd.data_ptr(), Wm, d)
    fwall, fev = timed_run(fc, yd[Wm:], K, d)
    S = len(plan)
    fc.close()
    full_cycle = {"stages_per_step": S, "particle_steps_per_s": N * K / fwall, "ms_per_step": fwall / K * 1e3,
                  "bytes_per_particle_step": S * B,
                  "hbm_frac_algorithmic": S * B * N / (fev / K) / 1e9 / HBM_PEAK_GBS}

    # -- island filter (AIRPF, Algorithms 4-7) ----------------------------------
    Mi = island_size(args, N)
    isl = make_island(Mi)
    isl.run(yd.data_ptr(), Wm, d)
    iwall, iev = timed_run(isl, yd[Wm:], K, d)
    isl.close()
    Bi = island_bytes(d, 4)
    island = {"island_size": Mi, "islands": N // Mi, "island_stages": (N // Mi).bit_length() - 1,
              "particle_steps_per_s": N * K / iwall, "ms_per_step": iwall / K * 1e3,
              "bytes_per_particle_step": Bi,
              "hbm_frac_algorithmic": Bi * N / (iev / K) / 1e9 / HBM_PEAK_GBS,
              "speedup_over_global": (N * K / iwall) / gvalue,
              "launches": ("within-island tile kernel, island stages (" +
                           ("blocks of 1024 islands, then one block" if N // Mi > 1024 else "one block") +
                           "), island gather")}

    # -- ESS-gated stages with a rotating start (Sections 1.2 and 6.4) ----------
    theta = 0.5
    ad = P.Filter(model, N, args.radix, seed=cfg["seed_pf"], history=K, stream=stream.cuda_stream,
                  ess_threshold=theta)
    ad.run(yd.data_ptr(), Wm, d)
    awall, aev = timed_run(ad, yd[Wm:], K, d)
    stages_run = [int(r["stage"]) for r in ad.history(K)]
    ad.close()
    s_mean = float(np.mean(stages_run)) if stages_run else 0.0
    Ba = adaptive_bytes(d, 4, s_mean)
    adaptive = {"ess_threshold": theta, "radix": args.radix, "stages_per_step_mean": s_mean,
                "particle_steps_per_s": N * K / awall, "ms_per_step": awall / K * 1e3,
                "bytes_per_particle_step": Ba,
                "hbm_frac_algorithmic": Ba * N / (aev / K) / 1e9 / HBM_PEAK_GBS,
                "launches_per_step": 3 + 2 * len(plan)}

    out = {
        "metric": "particle-steps/s + %HBM roofline, butterfly vs global BPF; p99 step latency",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} N=2^{N.bit_length() - 1} radix {args.radix}",
                   "n_particles": N, "state_dim": d, "radix": args.radix, "stages": plan,
                   "resampler": "multinomial", "steps_per_run": K, "observations": "device"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "pf_step_tile (fused butterfly step)",
                     "bytes_per_particle_step": B, "bytes_per_launch": launch_bytes,
                     "avg_launch_us": avg_launch_s * 1e6},
        "latency_us": {"p50": p50, "p99": p99, "mean": mean_us},
        "global_bpf": {"particle_steps_per_s": gvalue, "ms_per_step": gwall / K * 1e3,
                       "speedup_butterfly_over_global": value / gvalue,
                       "bytes_per_particle_step": Bg,
                       "hbm_frac_algorithmic": Bg * N / (gev / K) / 1e9 / HBM_PEAK_GBS,
                       "latency_us": {"p50": gp50, "p99": gp99}},
        "per_radix": per_radix,
        "full_cycle": full_cycle,
        "island": island,
        "adaptive": adaptive,
        "last_estimate": {"t": est["t"], "ess": est["ess"], "log_norm": est["log_norm"]},
    }
    if not args.no_batch and args.mode == "bench":
        out["batched"] = batched_bench(200, 5)
    if not args.no_serve and args.mode == "bench":
        out["serving"] = serving_bench(args.serve_window)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(model, N, args.radix, ys)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
