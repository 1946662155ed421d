"""Benchmark of the butterfly-interaction particle filter on one MI355X.

Headline workload: the stochastic volatility model (x' = 0.95 x + 0.25 z,
y = 0.6 exp(x / 2) e, x_0 from the stationary law), N = 2^24 particles,
radix 64 (stages 64, 64, 64, 64), multinomial resampling, FP32 states and
log-weights, FP64 log-normaliser; synthetic observations simulated from the
model (seed 3). One "step" is one filter time step over all N particles:
log-weight -> group resample -> gather -> propagate (+ estimate partials and
the deferred final reduction).

Printed (one JSON line): particle-steps/s of the headline with the
observations already in device memory, its p50/p99 step latency and the
roofline of the step kernel (algorithmic bytes / measured time against the
8 TB/s HBM peak); for the same model and N every radix in {32, 64, 256,
1024} and the global-resampling bootstrap filter (r = N), each with FP32 and
BF16 state storage, and the speedups over the global filter; the full-cycle,
island and ESS-gated variants; the 8-D linear-Gaussian model at N = 2^20
(radices 2, 4, 32, 64 and N); the batched and serving workloads; and the
FP64 oracle timed on the host as a baseline.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
       python bench.py --mode profile [--workload sv|lg8] [--radix R] [--dtype f32|bf16]
                       [--profile-island | --profile-adaptive | --profile-global]
                       (one filter's steps only, for rocprofv3)
       python bench.py --mode copybw   (device copy rate at 64 MiB to 4 GiB)
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
PROFILE_SUMMARY = {("lg8", 64, "f32"): os.path.join(ROOT, "profiles", "pf_step_tile_lg8_n2p20_r64.json"),
                   ("sv", 64, "f32"): os.path.join(ROOT, "profiles", "pf_step_tile_sv_n2p24_r64.json")}
STATE_BYTES = {"f32": 4, "bf16": 2, "f64": 8}
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
    """p50 / p99 / mean of single-step launches (HIP events around each),
    continuing the filter with the next observations ``yd[0 .. steps)``."""
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
    as many time steps of N particles as fit in about budget_s seconds (at
    least one)."""
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


def bf16_error(N: int = 1 << 16, radix: int = 64, T: int = 64, every: int = 8):
    """Error that state storage adds to each result of one step, FP32 and BF16
    against the FP64 instantiation of the same kernels (SV, N particles): at
    every `every`-th step of an FP64 trajectory, the FP64 cloud is rounded to
    the storage type, loaded into a filter of that type and stepped once;
    the FP64 filter takes the same step from the exact cloud. Largest error
    over the checkpoints: |d mean| / sd, |d var| / var, |d ESS| / ESS and
    |d log-normaliser increment|, with the Monte Carlo sd of the mean / sd
    (1 / sqrt(N ESS)) for scale."""
    import numpy as np
    import paper_1812_01502_amd as P
    import workloads as W
    model = W.sv_model()
    _, ys = W.simulate(model, T, seed=3)
    ref = P.Filter(model, N, radix, dtype="f64", seed=303)
    low = {dt: P.Filter(model, N, radix, dtype=dt, seed=303) for dt in ("f32", "bf16")}
    worst = {dt: dict(mean=0.0, var=0.0, ess=0.0, log_norm=0.0) for dt in low}
    mc = 0.0
    for t in range(T):
        if t % every == every - 1:
            x, w, tt, ln = ref.get_state()
            for dt, f in low.items():
                x32 = x.astype(np.float32)
                f.set_state(P.f32_to_bf16(x32) if dt == "bf16" else x32, w.astype(np.float32), t=tt, log_norm=0.0)
                f.step(ys[t])
        ref.step(ys[t])
        if t % every == every - 1:
            e0 = ref.estimate()
            sd = float(np.sqrt(e0["var"][0]))
            mc = max(mc, 1.0 / np.sqrt(N * e0["ess"]))
            dlam0 = e0["log_norm"] - ln
            for dt, f in low.items():
                e = f.estimate()
                wd = worst[dt]
                wd["mean"] = max(wd["mean"], abs(e["mean"][0] - e0["mean"][0]) / sd)
                wd["var"] = max(wd["var"], abs(e["var"][0] - e0["var"][0]) / e0["var"][0])
                wd["ess"] = max(wd["ess"], abs(e["ess"] - e0["ess"]) / e0["ess"])
                wd["log_norm"] = max(wd["log_norm"], abs(e["log_norm"] - dlam0))
    for f in [ref, *low.values()]:
        f.close()
    return {"workload": f"SV, N = {N}, radix {radix}, one step from the FP64 cloud at {T // every} steps "
                        f"of a {T}-step trajectory; reference: the FP64 kernels",
            "f32": worst["f32"], "bf16": worst["bf16"], "mc_sd_of_mean_over_sd": mc}


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


def serving_requests(rate: float, window_s: float, seed: int = 5):
    """Poisson arrivals (``rate`` streams/s over ``window_s``) of SV or 4-D LG
    streams (half each), N uniform over {2^12, 2^16, 2^20}, 50..500
    observations each, one observation per millisecond; observations are
    windows of one long simulated path per model."""
    import numpy as np
    import workloads as W
    from paper_1812_01502_amd.serving import StreamRequest
    rng = np.random.Generator(np.random.PCG64(seed))
    models = {"sv": W.sv_model(), "lg4": W.random_stable_lg(4, 5004)}
    Ns = [1 << 12, 1 << 16, 1 << 20]
    sim = {name: W.simulate(m, 20000, seed=seed)[1].reshape(20000, -1) for name, m in models.items()}
    t, reqs = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > window_s:
            break
        name = "sv" if rng.random() < 0.5 else "lg4"
        N = Ns[int(rng.integers(0, 3))]
        T = int(rng.integers(50, 501))
        o = int(rng.integers(0, 20000 - T))
        reqs.append(StreamRequest(stream_id=len(reqs), model=name, n_particles=N,
                                  observations=sim[name][o:o + T], arrival_s=t,
                                  seed=77 + len(reqs), cadence_s=1e-3))
    return models, reqs


def serving_bench(window_s: float = 5.0, rates=(250.0, 350.0, 500.0, 700.0, 1000.0, 2000.0), seed: int = 5):
    """The serving workload at several offered loads: continuous batching
    over re-bindable slots (admission by device footprint against a 24 GiB
    budget), per-observation latency from the observation's availability to
    its estimate in host memory. The offered load is the stream mix's
    particle-steps per second."""
    import numpy as np
    from paper_1812_01502_amd.serving import Server
    points = []
    for rate in rates:
        models, reqs = serving_requests(rate, window_s, seed)
        offered = sum(q.observations.shape[0] * q.n_particles for q in reqs) / window_s
        srv = Server(models, max_slots=1024, hbm_budget=24 << 30, radix=64, pipeline=3, max_substeps=8)
        _, st = srv.run(reqs, realtime=True, max_wall_s=240)
        srv.close()
        st.update(rate_streams_per_s=rate, offered_particle_steps_per_s=offered)
        points.append({k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()})
    return {"workload": f"Poisson arrivals over {window_s:g} s, SV or LG-4 (half each), N in 2^12/2^16/2^20, "
                        f"50..500 observations at 1 ms", "window_s": window_s, "load_points": points}


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


def load_traffic(path):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel sources; else None."""
    if path is None:
        return None
    try:
        with open(path) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    if prof.get("kernel_source_hash") != kernel_source_hash():
        return None
    return prof.get("hbm_bytes_per_launch")


class Legs:
    """Timed runs of single filters on one workload (model, N, observations
    in device memory): every leg creates a filter, runs W untimed steps,
    times K steps with HIP events around one pf_run, and closes it."""

    def __init__(self, name, cfg, N, K, Wm, stream):
        import torch
        import workloads as W
        self.name, self.cfg, self.N, self.K, self.Wm = name, cfg, N, K, Wm
        self.model = cfg["model"]
        self.d = self.model.d
        self.stream = stream
        # W + 2 K observations: warm-up, timed steps, then the latency steps
        _, self.ys = W.simulate(self.model, Wm + 2 * K, seed=cfg["seed_obs"])
        self.yd = torch.tensor(self.ys, dtype=torch.float32, device="cuda").contiguous()
        self.yd64 = torch.tensor(self.ys, dtype=torch.float64, device="cuda").contiguous()

    def make(self, radix, dtype="f32", **kw):
        import paper_1812_01502_amd as P
        return P.Filter(self.model, self.N, radix, dtype=dtype, seed=self.cfg["seed_pf"],
                        history=kw.pop("history", 4), stream=self.stream.cuda_stream, **kw)

    def y(self, dtype):
        return self.yd64 if dtype == "f64" else self.yd

    def time(self, flt, dtype="f32"):
        """(wall seconds, event seconds) of K steps after W warm-up steps."""
        yd = self.y(dtype)
        flt.run(yd.data_ptr(), self.Wm, self.d)
        return timed_run(flt, yd[self.Wm:], self.K, self.d)

    def leg(self, radix, dtype="f32", bytes_per=None, keep=False, **kw):
        """One timed filter: throughput, time per step, HBM fraction on the
        algorithmic bytes ``bytes_per`` per particle-step (default: the fused
        butterfly step, or the global path's for r >= N)."""
        flt = self.make(radix, dtype, **kw)
        info = flt.info()
        wall, ev = self.time(flt, dtype)
        s = STATE_BYTES[dtype]
        if bytes_per is None:
            bytes_per = algorithmic_bytes(self.d, s, "global" if radix >= self.N else "butterfly")
        out = dict(particle_steps_per_s=self.N * self.K / wall, ms_per_step=wall / self.K * 1e3,
                   avg_step_us=ev / self.K * 1e6, bytes_per_particle_step=bytes_per,
                   hbm_frac=bytes_per * self.N / (ev / self.K) / 1e9 / HBM_PEAK_GBS,
                   stages=info["stages"])
        if keep:
            return out, flt
        flt.close()
        return out, None


def safe(fn, *a, **kw):
    """Run one bench leg; a failure is recorded in the output instead of
    ending the run."""
    try:
        return fn(*a, **kw)
    except Exception as e:   # noqa: BLE001 - reported in the JSON line
        return {"error": f"{type(e).__name__}: {e}"}


def variants(L: Legs, radix: int, island_M: int):
    """Full-cycle, island and ESS-gated filters on one workload."""
    import numpy as np
    d, N, K = L.d, L.N, L.K
    B = algorithmic_bytes(d, 4, "butterfly")
    out = {}

    def full():
        fc, _ = L.leg(radix, bytes_per=None, full_cycle=True)
        S = len(fc["stages"])
        fc.update(stages_per_step=S, bytes_per_particle_step=S * B, hbm_frac=fc["hbm_frac"] * S)
        return fc
    out["full_cycle"] = safe(full)

    def island():
        Bi = island_bytes(d, 4)
        r, _ = L.leg(2, bytes_per=Bi, island=island_M)
        r.update(island_size=island_M, islands=N // island_M, island_stages=(N // island_M).bit_length() - 1,
                 launches=("within-island tile kernel, island stages (" +
                           ("blocks of 1024 islands, then one block" if N // island_M > 1024 else "one block") +
                           "), island gather"))
        return r
    out["island"] = safe(island)

    def adaptive():
        theta = 0.5
        flt = L.make(radix, history=K, ess_threshold=theta)
        wall, ev = L.time(flt)
        stages_run = [int(r["stage"]) for r in flt.history(K)]
        flt.close()
        s_mean = float(np.mean(stages_run)) if stages_run else 0.0
        Ba = adaptive_bytes(d, 4, s_mean)
        return dict(ess_threshold=theta, radix=radix, stages_per_step_mean=s_mean,
                    particle_steps_per_s=N * K / wall, ms_per_step=wall / K * 1e3,
                    bytes_per_particle_step=Ba, hbm_frac=Ba * N / (ev / K) / 1e9 / HBM_PEAK_GBS,
                    launches_per_step=3 + 2 * len(L.make(radix).info()["stages"]))
    out["adaptive"] = safe(adaptive)
    return out


def copy_bandwidth(sizes_mib=(64, 128, 256, 512, 1024, 4096), reps=20):
    """Device-to-device copy rate (bytes read + bytes written per second) of
    torch's copy at several sizes, with HIP events around ``reps`` copies
    after two untimed ones. Sizes above the 256 MB Infinity Cache give the
    practical HBM ceiling that the step kernels are compared with."""
    import torch
    out = []
    for mib in sizes_mib:
        n = mib << 18   # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        out.append({"mib": mib, "us_per_copy": us, "gb_per_s": 2 * n * 4 / us / 1e3})
        del src, dst
    return out


def profile_mode(args, L: Legs):
    """One filter's warm-up and timed steps (for rocprofv3), then a plain copy
    of known size (counter calibration)."""
    import torch
    rs = args.resampler
    if args.profile_island:
        flt = L.make(2, args.dtype, island=island_size(args, L.N), resampler=rs)
    elif args.profile_adaptive:
        flt = L.make(args.radix, args.dtype, ess_threshold=0.5, resampler=rs)
    elif args.profile_global:
        flt = L.make(L.N, args.dtype, resampler=rs)
    else:
        flt = L.make(args.radix, args.dtype, resampler=rs)
    wall, ev_s = L.time(flt, args.dtype)
    flt.close()
    src = torch.empty(1 << 27, dtype=torch.float32, device="cuda")   # 512 MiB
    src.fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": True, "copy_bytes": src.numel() * 4, "warmup": L.Wm, "steps": L.K,
                      "avg_step_us": ev_s / L.K * 1e6}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed steps of every filter before its timed steps")
    ap.add_argument("--radix", type=int, default=64, help="radix of the headline (and of --mode profile)")
    ap.add_argument("--dtype", choices=["f32", "bf16"], default="f32", help="--mode profile: state storage")
    ap.add_argument("--resampler", choices=["multinomial", "systematic"], default="multinomial",
                    help="--mode profile: resampler")
    ap.add_argument("--mode", choices=["bench", "profile", "copybw"], default="bench",
                    help="copybw: the device-to-device copy rate at several sizes (the practical HBM ceiling)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=["sv", "lg8"], default="sv",
                    help="--mode profile: sv (stochastic volatility, N = 2^24) or lg8 (8-D LG, N = 2^20)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-filters section")
    ap.add_argument("--batch-only", action="store_true", help="print only the batched-filters section")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--serve-only", action="store_true", help="print only the serving section")
    ap.add_argument("--no-lg8", action="store_true", help="skip the 8-D LG section")
    ap.add_argument("--island", type=int, default=0, help="island size of the island-filter sections")
    ap.add_argument("--profile-island", action="store_true",
                    help="--mode profile: run the island filter instead of the butterfly filter")
    ap.add_argument("--profile-adaptive", action="store_true",
                    help="--mode profile: run the ESS-gated filter (theta 0.5) instead")
    ap.add_argument("--profile-global", action="store_true",
                    help="--mode profile: run the global bootstrap filter (r = N) instead")
    ap.add_argument("--serve-window", type=float, default=5.0, help="arrival window of each serving load point (s)")
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
    if args.mode == "copybw":
        print(json.dumps({"copy_bandwidth": copy_bandwidth()}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batched": batched_bench(200, 5)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serving_bench(args.serve_window)}), flush=True)
        return
    K, Wm = args.steps, args.warmup
    stream = torch.cuda.current_stream()
    if args.mode == "profile":
        cfg = W.config("c3" if args.workload == "sv" else "c2")
        profile_mode(args, Legs(args.workload, cfg, cfg["N"], K, Wm, stream))
        return

    # -- 8-D LG, N = 2^20 (run first: the GPU's clocks settle meanwhile) ------
    lg8 = None
    if not args.no_lg8:
        c2 = W.config("c2")
        L2 = Legs("lg8", c2, c2["N"], K, Wm, stream)
        lg8 = {"workload": "8-D LG (A = 0.9 I + 0.05 O, Q = I, H = I, R = 0.5 I), N = 2^20, FP32",
               "per_radix": {}}
        for r in (2, 4, 32, 64):
            lg8["per_radix"][str(r)] = safe(lambda r=r: L2.leg(r)[0])
        g2 = safe(lambda: L2.leg(L2.N)[0])
        lg8["global_bpf"] = g2
        if "particle_steps_per_s" in g2:
            for r, v in lg8["per_radix"].items():
                if "particle_steps_per_s" in v:
                    v["speedup_over_global"] = v["particle_steps_per_s"] / g2["particle_steps_per_s"]
        lg8.update(variants(L2, 64, args.island or 1024))
        del L2

    # -- stochastic volatility, N = 2^24: every radix, FP32 and BF16 ----------
    c3 = W.config("c3")
    L3 = Legs("sv", c3, c3["N"], K, Wm, stream)
    N, d = L3.N, L3.d
    sv = {"workload": "stochastic volatility, N = 2^24", "per_radix": {}, "global_bpf": {}}
    for dt in ("f32", "bf16"):
        sv["global_bpf"][dt] = safe(lambda dt=dt: L3.leg(N, dt)[0])
        for r in (32, 256, 1024) + ((64,) if dt == "bf16" else ()):
            sv["per_radix"][f"{r} {dt}"] = safe(lambda r=r, dt=dt: L3.leg(r, dt)[0])
    # systematic resampling: monotone draws, so the global filter's reads of
    # the CDF and its gather are near-sequential
    sv["systematic"] = {"64 f32": safe(lambda: L3.leg(64, "f32", resampler="systematic")[0]),
                        "global f32": safe(lambda: L3.leg(N, "f32", resampler="systematic")[0])}
    sv.update(variants(L3, 64, args.island or 4096))

    # -- the headline: radix 64, FP32 ------------------------------------------
    head, flt = L3.leg(args.radix, "f32", keep=True)
    sv["per_radix"][f"{args.radix} f32"] = head
    p50, p99, mean_us = per_step_latency(flt, L3.yd[Wm + K:], K, d)
    est = flt.estimate()
    flt.close()
    for key, v in sv["per_radix"].items():
        g = sv["global_bpf"].get(key.split()[1], {})
        if "particle_steps_per_s" in v and "particle_steps_per_s" in g:
            v["speedup_over_global"] = v["particle_steps_per_s"] / g["particle_steps_per_s"]
    B = algorithmic_bytes(d, 4, "butterfly")
    launch_bytes = B * N
    avg_launch_s = head["avg_step_us"] * 1e-6     # one step kernel per step
    achieved = launch_bytes / avg_launch_s / 1e9
    traffic = load_traffic(PROFILE_SUMMARY.get(("sv", args.radix, "f32")))
    gf = sv["global_bpf"].get("f32", {})
    gs = sv.get("systematic", {}).get("global f32", {})

    out = {
        "metric": "particle-steps/s + %HBM roofline, butterfly vs global BPF; p99 step latency",
        "value": head["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"stochastic volatility (x' = 0.95 x + 0.25 z, y = 0.6 e^(x/2) e), "
                               f"N = 2^{N.bit_length() - 1}, radix {args.radix}, FP32 states",
                   "n_particles": N, "state_dim": d, "radix": args.radix, "stages": head["stages"],
                   "resampler": "multinomial", "steps_per_run": K, "observations": "device"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "pf_step_tile (fused butterfly step)",
                     "bytes_per_particle_step": B, "bytes_per_launch": launch_bytes,
                     "avg_launch_us": avg_launch_s * 1e6},
        "latency_us": {"p50": p50, "p99": p99, "mean": mean_us},
        "speedup_butterfly_over_global": (head["particle_steps_per_s"] / gf["particle_steps_per_s"]
                                          if "particle_steps_per_s" in gf else None),
        # against the faster global filter: systematic resampling by offspring ranges
        "speedup_butterfly_over_global_systematic": (
            head["particle_steps_per_s"] / gs["particle_steps_per_s"] if "particle_steps_per_s" in gs else None),
        "sv": sv,
        "lg8": lg8,
        "last_estimate": {"t": est["t"], "ess": est["ess"], "log_norm": est["log_norm"],
                          "mean": float(est["mean"][0])},
    }
    out["bf16_error"] = safe(bf16_error)
    if not args.no_batch:
        out["batched"] = safe(batched_bench, 200, 5)
    if not args.no_serve:
        out["serving"] = safe(serving_bench, args.serve_window)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(L3.model, N, args.radix, L3.ys)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
