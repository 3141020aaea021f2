"""Throughput of the noisy D2Q9 hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5_4096]
                    [--storage f32|bf16|f16] [--no-cpu-baseline] [--no-forms]

One benchmark step is one pass of the whole path on the workload: ten fused
collide+noise+stream updates of every site and one correlator sample (field
extraction with the FP64 conservation sums of the sampled state, 2-D
transforms, FP64 accumulation of the fifteen products).  The library runs
each sample beside the next ten updates (on a second stream); the handle's
flush call, which enqueues a sample still waiting for steps and adds the
products of the samples whose spectra are stashed, and the device
synchronisation close the timed region, which opens with no sample owed: the
whole work of exactly K samples runs inside it.  W untimed steps, then K
timed steps.  `value` is site updates per
second (GLUPS) over the timed region, inputs resident in HBM.

The JSON line also carries
  roofline      the step kernel (dominant): algorithmic bytes per launch
                (9 reads + 9 writes per site update, times the updates of
                one launch: two per site for the time-blocked kernel, which
                moves the state once for both) over its average duration,
                measured with a HIP event pair around each launch of every
                fourth benchmark step on the stream it runs on, within the
                timed region (so while the sample shares the device;
                `launches_timed` counts them; `isolated` repeats the figures
                for the kernel alone);
                HBM traffic per launch from rocprofv3 counters when a
                summary for the current kernel source is committed, and the
                rate it implies (measured_GBs); step_kernel_glups_isolated
                times the step kernel alone after the timed region, and
                sample_ms is what a period takes beyond ten isolated steps;
  cpu_baseline  the FP64 oracle on a bounded sample of the same workload,
                over every CPU the process may use (value, cores) and on one
                thread (single_core_value), with the host's CPU model;
  forms         step-kernel rates of the other storage formats and of the
                noise-free step (the paper's ghost-noise overhead), and the
                batched forms (96 x 512^2 Galilean-invariance sweep, 64
                uneven lattices) through graph-replayed sampling periods,
                and the other velocity sets (D3Q15 at 256^3 with its
                correlators, D1Q3 at 2^26 sites).
Every handle's step-kernel launch shape is chosen by the library's autotuner
before timing: on whole sampling periods (flb_autotune_path) for the
headline workload and the batched forms, on the step kernel alone
(flb_autotune) for the storage forms' step rates.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "noisy D2Q9 GLUPS and % of HBM peak, FP32/batched vs plain, at matched S(k)"
HBM_PEAK_GBS = 8000.0
SAMPLE_EVERY = 10
# samples per read-modify-write pass of the FP64 correlator sums in the
# library (the others keep their spectra until then)
ACCUMULATE_EVERY = 32
LAUNCH_TIMING_EVERY = 4  # benchmark steps per step whose launches are timed
STEP_KERNEL = "step_kernel"


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("flb_step.hip", "flb_device.h", "flb_internal.h"):
        with open(os.path.join(ROOT, "paper_1010_1233_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def shape_key(workload, storage, shape, blocking=(1, 64)):
    """Key of a launch shape: one-step kernels by threads x sites, the
    two-step kernel by its tile width."""
    tw, sites, nt = shape
    if blocking[0] >= 2:
        return f"{workload}/{storage}/step{blocking[0]}_{blocking[1]}/nt{int(bool(nt))}"
    return f"{workload}/{storage}/{tw}x{sites}/nt{int(bool(nt))}"


KERNEL_OF_STEPS = {1: STEP_KERNEL, 2: "step2_kernel", 3: "step3_kernel"}


def launch_figures(g, sites, step_ms, steps=None):
    """The dominant kernel's launch: which kernel, steps per launch, its
    duration and its algorithmic bytes = 18 values per site update (9 loads
    + 9 stores) x the site updates of one launch.  The two- and three-step
    kernels do two or three updates per site and launch on one read and one
    write of the state, so their algorithmic rate can exceed what HBM moves
    (see the measured traffic)."""
    if steps is None:
        steps = g.time_blocking()[0]
    bpv = g.storage_info()[1]
    launch_ms = steps * step_ms
    algo = 18 * bpv * sites * steps
    return {"kernel": KERNEL_OF_STEPS[steps],
            "steps_per_launch": steps, "avg_launch_ms": launch_ms,
            "algorithmic_bytes_per_launch": algo,
            "achieved_GBs": algo / (launch_ms * 1e-3) / 1e9}


def counter_entry(workload, storage, shape, blocking=(1, 64)):
    """This launch shape's entry of the committed counter summary (HBM bytes
    per step-kernel launch, VALU instructions per site update), or {}
    when it is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return {}
    e = d.get(shape_key(workload, storage, shape, blocking))
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return {}
    return e


def measured_traffic(workload, storage, shape, blocking=(1, 64)):
    """HBM bytes per step-kernel launch of this launch shape from the
    committed counter summary, or None (see counter_entry)."""
    return counter_entry(workload, storage, shape, blocking).get("bytes_per_launch")


def sweep_shapes(flb, workloads, name, storage, steps=5):
    """Runs every step-kernel launch shape for a few steps (no timing): the
    workload for per-shape hardware-counter runs."""
    g, c = make_lattice(flb, workloads, name, storage)
    g.thermalize()
    for tw in (64, 128, 256):
        for sites in (1, 2, 4):
            for nt in (0, 1):
                g.set_step_config(tw, sites, nt)
                g.step(steps)
    for blocking in (2, 3):
        for tile2 in (32, 64, 128):
            for nt in (0, 1):
                g.set_step_config(256, 1, nt)
                g.set_time_blocking(blocking, tile2)
                g.step(blocking * steps)
    g.set_time_blocking(1, 64)
    g.synchronize()
    print(f"sweep-shapes: {name} {storage}: 18 one-step shapes x {steps} steps, "
          f"6 two-step and 6 three-step shapes x {steps} launches", flush=True)


def make_lattice(flb, workloads, name, storage):
    c = workloads.CONFIGS[name]
    g = flb.Lattice(c["nx"], c["ny"], c["tau"], c["theta"], rho0=c["rho0"], u0=c["u0"],
                    seed=c["seed"], storage=storage)
    return g, c


def time_step_kernel(torch, g, stream, n):
    """Average duration (ms) of n back-to-back step launches on `stream`."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.step(n)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / n


def steady_step_ms(torch, g, stream, n=60, warm=120, reps=3):
    """Step time (ms) of a handle alone: `warm` untimed steps (the device
    leaves the power state of whatever ran before), then the fastest of
    `reps` runs of n steps."""
    time_step_kernel(torch, g, stream, warm)
    return min(time_step_kernel(torch, g, stream, n) for _ in range(reps))


# VALU issue: 256 CUs x 2.4 GHz, one wave-level (64-lane) VALU instruction
# per CU and cycle (four SIMDs of 16 lanes)
VALU_ISSUE_PER_S = 256 * 2.4e9


def valu_issue_frac(valu_per_update, updates_per_launch, launch_ms):
    """Time the launch's VALU instructions need at the issue rate over its
    duration (None without the counters' figure)."""
    if valu_per_update is None:
        return None
    return valu_per_update * updates_per_launch / 64 / VALU_ISSUE_PER_S / (launch_ms * 1e-3)


def copy_GBs(torch, stream, nbytes, n=20, reps=3):
    """The device copy's practical rate (read + write bytes per second) over
    nbytes each way, on `stream`: the fastest of `reps` runs of n copies."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = 1e30
    with torch.cuda.stream(stream):
        for _ in range(3):
            b.copy_(a)
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(n):
                b.copy_(a)
            e1.record(stream)
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / n)
    del a, b
    return 2 * nbytes / (best * 1e-3) / 1e9


def plain_path_ms(torch, g, stream, n=ACCUMULATE_EVERY, warm=16):
    """Whole-path time (ms) per benchmark step of one handle with the timed
    region's calls (SAMPLE_EVERY steps and a sample, plain calls): `warm`
    untimed benchmark steps and a flush, then n timed ones ending with the
    flush of their stashed samples."""
    with torch.cuda.stream(stream):
        for _ in range(warm):
            g.step(SAMPLE_EVERY)
            g.accumulate()
        g.flush_correlators()
        g.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            g.step(SAMPLE_EVERY)
            g.accumulate()
        g.flush_correlators()
        g.synchronize()
        e1.record(stream)
        e1.synchronize()
    return e0.elapsed_time(e1) / n


def batched_form(torch, flb, stream, specs, storage, periods=ACCUMULATE_EVERY):
    """Whole path (graph-replayed periods of SAMPLE_EVERY steps + a sample)
    and step-only rates of one batched handle."""
    # the captured periods depend on the buffer parity and on how many of the
    # samples of an accumulation cycle are stashed: a whole number of cycles
    # starts the timed run where the warm-up started, so that it replays
    # graphs the warm-up captured
    assert periods % ACCUMULATE_EVERY == 0
    b = flb.Lattice.batch(specs, seed=3, storage=storage)
    b.set_stream(stream)
    b.thermalize()
    shape, _ = b.autotune_path(50, SAMPLE_EVERY)
    sites = sum(s["nx"] * s["ny"] for s in specs)
    b.run(periods * SAMPLE_EVERY, SAMPLE_EVERY)  # capture the graphs
    b.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.run(periods * SAMPLE_EVERY, SAMPLE_EVERY)
    b.synchronize()  # enqueues the last sample and waits for it
    e1.record(stream)
    e1.synchronize()
    ms_period = e0.elapsed_time(e1) / periods
    step_ms = steady_step_ms(torch, b, stream)
    lf = launch_figures(b, sites, step_ms)
    shape = list(shape) + [list(b.time_blocking())]
    tiles = b.lattice_tiles()
    b.close()
    return {"lattices": len(specs), "sites": sites, "launch_shape": shape,
            # lattices per two-step tile width (the tuner's choice per size class)
            "lattice_tiles": {str(w): tiles.count(w) for w in sorted(set(tiles))},
            "path_glups": SAMPLE_EVERY * sites / (ms_period * 1e-3) / 1e9,
            "step_glups": sites / (step_ms * 1e-3) / 1e9,
            "steps_per_launch": lf["steps_per_launch"],
            "step_achieved_GBs": lf["achieved_GBs"],
            "sample_ms": max(ms_period - SAMPLE_EVERY * step_ms, 0.0)}


def shard_form(torch, flb, workloads, stream, name, storage, strips=8):
    """One GPU's share of the workload's lattice split into `strips` x-strips
    (nx / strips x ny sites, the workload's parameters, periodic): step rate
    and whole-path rate with the strip's own sample."""
    c = workloads.CONFIGS[name]
    nx, ny = c["nx"] // strips, c["ny"]
    g = flb.Lattice(nx, ny, c["tau"], c["theta"], rho0=c["rho0"], u0=c["u0"], seed=c["seed"],
                    storage=storage)
    g.set_stream(stream)
    g.thermalize()
    shape, _ = g.autotune_path(50, SAMPLE_EVERY)
    step_ms = steady_step_ms(torch, g, stream)
    pms = plain_path_ms(torch, g, stream)
    out = {"sites": nx * ny, "sides": [nx, ny],
           "launch_shape": list(shape) + [list(g.time_blocking())],
           "step_glups": nx * ny / (step_ms * 1e-3) / 1e9,
           "path_glups": SAMPLE_EVERY * nx * ny / (pms * 1e-3) / 1e9,
           "sample_ms": max(pms - SAMPLE_EVERY * step_ms, 0.0)}
    g.close()
    return out


def velocity_set_form(torch, flb, stream, model, sides, sample=True, periods=5):
    """Step (and, where the sides allow correlators, whole-path) rates of one
    lattice of another velocity set: FP32 deviations, Q loads + Q stores per
    site."""
    D, _, w, _ = flb.dq_tables(model)
    Q = len(w)
    tau = [1.0] * (D + 1) + [0.8] * (D * (D + 1) // 2) + [1.0] * (Q - 1 - D - D * (D + 1) // 2)
    g = flb.DqLattice(model, sides, tau, 1e-4, u0=[0.05, 0.0, 0.0][:D], seed=7)
    g.set_stream(stream)
    g.thermalize()
    sites = g.sides[0] * g.sides[1] * g.sides[2]
    g.step(50)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    g.step(20)
    e1.record(stream)
    e1.synchronize()
    step_ms = e0.elapsed_time(e1) / 20
    out = {"sites": sites, "bytes_per_site": 2 * Q * 4,
           "step_glups": sites / (step_ms * 1e-3) / 1e9,
           "step_achieved_GBs": 2 * Q * 4 * sites / (step_ms * 1e-3) / 1e9}
    if sample:
        g.run(2 * SAMPLE_EVERY, SAMPLE_EVERY)
        e0.record(stream)
        g.run(periods * SAMPLE_EVERY, SAMPLE_EVERY)
        e1.record(stream)
        e1.synchronize()
        ms_period = e0.elapsed_time(e1) / periods
        out["path_glups"] = SAMPLE_EVERY * sites / (ms_period * 1e-3) / 1e9
        out["sample_ms"] = max(ms_period - SAMPLE_EVERY * step_ms, 0.0)
    g.close()
    return out


def cpu_baseline(workloads, name, side=1024):
    """The oracle (FP64, as it stands) on a bounded sample of the same
    workload: its parameters on side^2 lattices, ten steps and one
    correlator sample per lattice (one benchmark step), first on one thread,
    then on every CPU the process may use with one lattice per thread
    (ctypes releases the interpreter lock during the oracle's calls, so the
    threads run in parallel).  Lattices are set up before the clock starts."""
    import threading

    import oracle
    c = workloads.CONFIGS[name]
    nx, ny = min(c["nx"], side), min(c["ny"], side)
    V = nx * ny
    oracle.tables()  # the oracle's constant tables, set up once before any thread

    def lattice(i):
        return oracle.Lattice(nx, ny, c["tau"], c["theta"], rho0=c["rho0"], u0=c["u0"],
                              seed=c["seed"], stream_id=i)

    def work(L):
        L.step(SAMPLE_EVERY)
        L.sample()

    L = lattice(0)
    t0 = time.perf_counter()
    work(L)
    dt1 = time.perf_counter() - t0
    del L
    host = host_cpu()
    n = max(1, int(host["cpus_available"] or 1))
    lats = [lattice(i) for i in range(n)]
    threads = [threading.Thread(target=work, args=(x,)) for x in lats]
    t0 = time.perf_counter()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    dtn = time.perf_counter() - t0
    del lats
    return {"value": n * SAMPLE_EVERY * V / dtn / 1e9, "unit": "GLUPS", "cores": n,
            "kind": "oracle",
            "single_core_value": SAMPLE_EVERY * V / dt1 / 1e9,
            "sample": f"{SAMPLE_EVERY} steps + 1 correlator sample of a {nx}x{ny} lattice with "
                      f"the workload's parameters, FP64: on one thread ({dt1:.1f} s), then one "
                      f"such lattice on each of {n} threads at once ({dtn:.1f} s)",
            "host": host}


def sample_only(torch, flb, workloads, names, n=2 * ACCUMULATE_EVERY, warm=ACCUMULATE_EVERY):
    """Correlator samples of a fixed (thermal) state enqueued back to back,
    nothing beside them: ms per sample for each named workload (c5_4096,
    batched_gi_96x512, batched_uneven_64), the sums' read-modify-writes
    included (a whole number of accumulation cycles, then a flush)."""
    c = workloads.CONFIGS["c5_4096"]
    specs = {"c5_4096": [dict(nx=c["nx"], ny=c["ny"], tau=c["tau"], theta=c["theta"],
                              u0=c["u0"])],
             "batched_gi_96x512": workloads.gi_sweep_specs(),
             "batched_uneven_64": workloads.uneven_batch_specs()}
    out = {}
    stream = torch.cuda.Stream()
    for name in names:
        b = flb.Lattice.batch(specs[name], seed=3)
        b.set_sample_overlap(False)
        b.set_stream(stream)
        b.thermalize()
        for _ in range(warm):
            b.accumulate()
        b.flush_correlators()
        b.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            b.accumulate()
        b.flush_correlators()
        e1.record(stream)
        e1.synchronize()
        out[name] = {"sample_ms": e0.elapsed_time(e1) / n, "samples": n}
        print(f"sample-only: {name} {out[name]}", flush=True)
        b.close()
    return out


def host_cpu():
    """The host's CPU model and the number of CPUs this process may use."""
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        ncpu = os.cpu_count()
    return {"model": model, "cpus_available": ncpu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c5_4096")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--sweep-shapes", action="store_true",
                    help="only run every step-kernel launch shape briefly (for counter runs)")
    ap.add_argument("--velocity-sets", action="store_true",
                    help="only time the other velocity sets (D3Q15 at 256^3 with its "
                         "correlators, D1Q3 at 2^26 sites) and print their figures")
    ap.add_argument("--sample-only", nargs="*", default=None, metavar="WORKLOAD",
                    help="only time correlator samples alone (no steps beside them) on the "
                         "named workloads (default: c5_4096 batched_gi_96x512 "
                         "batched_uneven_64) and print their figures")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 603,979,776 bytes device to device three times "
                         "(the known-size reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (independent "
              "lattices would shard across GPUs with one final all-reduce of the FP64 sums). "
              "Use --gpus 1.", file=sys.stderr)
        return 2

    import torch

    import paper_1010_1233_amd as flb
    from paper_1010_1233_amd import workloads

    assert torch.cuda.is_available(), "no GPU visible"
    if args.copy_calibration:
        a = torch.ones(9 * 4096 * 4096, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copy-calibration: 3 x {a.numel() * 4} bytes", flush=True)
        # the same copy timed: the runtime's practical copy bandwidth
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 20
        print(f"copy-calibration: device copy {2 * a.numel() * 4 / (ms * 1e-3) / 1e9:.0f} GB/s "
              f"(read + write) over {a.numel() * 4} bytes", flush=True)
        return 0
    if args.sweep_shapes:
        sweep_shapes(flb, workloads, args.workload, args.storage)
        return 0
    if args.sample_only is not None:
        names = args.sample_only or ["c5_4096", "batched_gi_96x512", "batched_uneven_64"]
        print(json.dumps(sample_only(torch, flb, workloads, names)), flush=True)
        return 0
    if args.velocity_sets:
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            out = {"d3q15_256x256x256": velocity_set_form(torch, flb, stream, "D3Q15",
                                                          (256, 256, 256)),
                   "d1q3_67108864": velocity_set_form(torch, flb, stream, "D1Q3", (1 << 26,),
                                                      sample=False)}
        print(json.dumps(out), flush=True)
        return 0
    stream = torch.cuda.Stream()
    g, c = make_lattice(flb, workloads, args.workload, args.storage)
    g.set_stream(stream)
    V = c["nx"] * c["ny"]
    print(f"bench: {args.workload} {c['nx']}x{c['ny']} storage={args.storage} "
          f"step config={g.step_config()}", file=sys.stderr, flush=True)
    g.thermalize()
    # the launch shape that makes the whole path fastest (the shapes nearly
    # tied alone, timed on periods with the sample beside the steps)
    tuned, _ = g.autotune_path(50, SAMPLE_EVERY)
    blocking = g.time_blocking()
    print(f"bench: autotuned step config {tuned}, steps per launch {blocking}", file=sys.stderr,
          flush=True)
    cons0 = g.conservation()

    def bench_step():
        g.step(SAMPLE_EVERY)
        g.accumulate()

    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            bench_step()
        # the warm-up's stashed samples are added before the window opens, so
        # that the window holds the whole work of exactly its own samples
        g.flush_correlators()
        g.synchronize()
        torch.cuda.synchronize()
        # HIP event pairs around the step-kernel launches of every
        # LAUNCH_TIMING_EVERY-th benchmark step of the timed region (an event
        # pair around every launch cost about 20 us per benchmark step)
        t0 = time.perf_counter()
        for i in range(args.steps):
            timed = i % LAUNCH_TIMING_EVERY == 0
            if timed:
                g.set_launch_timing(True)
            g.step(SAMPLE_EVERY)
            if timed:
                g.set_launch_timing(False)
            g.accumulate()
        # enqueues the last sample and the products of the stashed ones
        g.flush_correlators()
        g.synchronize()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        kinds = g.launch_timing_kinds()

    # launches of 1, 2 and 3 steps (with three steps per launch a period of
    # ten steps is 3 + 3 + 2 + 2); the roofline takes the kind that took the
    # most time
    steps_timed = -(-args.steps // LAUNCH_TIMING_EVERY)
    assert sum((q + 1) * n for q, (n, _) in enumerate(kinds)) == steps_timed * SAMPLE_EVERY, kinds
    n_launches = sum(n for n, _ in kinds)
    step_ms = sum(ms for _, ms in kinds) / (steps_timed * SAMPLE_EVERY)
    qd = max(range(3), key=lambda q: kinds[q][1])
    ms_per_step = elapsed * 1e3 / args.steps
    value = args.steps * SAMPLE_EVERY * V / elapsed / 1e9
    launch = launch_figures(g, V, kinds[qd][1] / kinds[qd][0] / (qd + 1), steps=qd + 1)
    achieved = launch["achieved_GBs"]
    traffic = measured_traffic(args.workload, args.storage, tuned, blocking)
    valu = counter_entry(args.workload, args.storage, tuned, blocking).get("valu_insts_per_update")
    drift = float(abs(g.sample_conservation()[0] - cons0[0]))

    # correlator sanity (matched S(k)): k-averaged S(rho) over the run
    S = g.read_normalized()
    s_rho_mean = float(S["S_rho"][1:, 1:].mean())

    # the step kernel alone (nothing sampled beside it), after enough
    # untimed steps that the device has left the power state of the idle
    # host-side read above
    with torch.cuda.stream(stream):
        # 120 steps: whole launches of the dominant kind
        iso_ms = steady_step_ms(torch, g, stream, n=120, warm=240)
    iso = launch_figures(g, V, iso_ms)
    # the device copy of one population buffer (the bytes one step moves at
    # the algorithmic count): the practical ceiling next to 8 TB/s
    copy_rate = copy_GBs(torch, stream, 9 * V * g.storage_info()[1])

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"D2Q9 {c['nx']}x{c['ny']} periodic, {args.storage} storage, "
                               f"rho0={c['rho0']}, u0={tuple(c['u0'])}, tau_shear={c['tau'][3]}, "
                               f"kT={c['theta']}, thermal start, correlators every "
                               f"{SAMPLE_EVERY} steps",
                   "sites": V, "lb_steps_per_bench_step": SAMPLE_EVERY,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": launch["kernel"],
                     "steps_per_launch": launch["steps_per_launch"],
                     "algorithmic_bytes_per_launch": launch["algorithmic_bytes_per_launch"],
                     "avg_launch_ms": launch["avg_launch_ms"],
                     "launches_timed": n_launches,
                     "launches_of_kernel": kinds[qd][0],
                     "launch_shape": list(tuned) + [list(blocking)],
                     "measured_GBs": (None if traffic is None else
                                      traffic / (launch["avg_launch_ms"] * 1e-3) / 1e9),
                     "measured_frac": (None if traffic is None else
                                       traffic / (launch["avg_launch_ms"] * 1e-3) / 1e9
                                       / HBM_PEAK_GBS),
                     # VALU instructions (per lane) per site update, from
                     # the counters (SQ_INSTS_VALU x 64 / updates per launch)
                     "valu_insts_per_update": valu,
                     # the same instructions at the VALU issue rate over the
                     # launch's duration: the kernel's other bound
                     "valu_issue_frac": valu_issue_frac(valu, V * launch["steps_per_launch"],
                                                        launch["avg_launch_ms"]),
                     "copy": {"bytes_each_way": 9 * V * g.storage_info()[1],
                              "GBs": copy_rate, "achieved_over_copy": achieved / copy_rate,
                              "measured_over_copy": (None if traffic is None else
                                                     traffic / (launch["avg_launch_ms"] * 1e-3)
                                                     / 1e9 / copy_rate)},
                     "isolated": {"avg_launch_ms": iso["avg_launch_ms"],
                                  "achieved": iso["achieved_GBs"],
                                  "frac": iso["achieved_GBs"] / HBM_PEAK_GBS,
                                  "measured_GBs": (None if traffic is None else
                                                   traffic / (iso["avg_launch_ms"] * 1e-3) / 1e9),
                                  "valu_issue_frac": valu_issue_frac(
                                      valu, V * iso["steps_per_launch"], iso["avg_launch_ms"])}},
        "step_kernel_glups": V / (step_ms * 1e-3) / 1e9,
        "step_kernel_glups_isolated": V / (iso_ms * 1e-3) / 1e9,
        "sample_ms": max(ms_per_step - SAMPLE_EVERY * iso_ms, 0.0),
        # every timed sample's transforms and its share of the FP64 sums'
        # read-modify-write passes (one per ACCUMULATE_EVERY samples, plus one
        # for the remainder) ran inside the window
        "samples_timed": args.steps,
        "accumulations_timed": -(-args.steps // ACCUMULATE_EVERY),
        "mass_drift": drift,
        "S_rho_kmean": s_rho_mean,
    }

    if not args.no_forms:
        forms = {}
        with torch.cuda.stream(stream):
            for st in ("f32", "bf16", "f16"):
                if st == args.storage:
                    continue
                h, _ = make_lattice(flb, workloads, args.workload, st)
                h.set_stream(stream)
                h.thermalize()
                shape, _ = h.autotune(50)
                ms = steady_step_ms(torch, h, stream)
                lf = launch_figures(h, V, ms)
                pms = plain_path_ms(torch, h, stream)
                forms[st] = {"step_glups": V / (ms * 1e-3) / 1e9,
                             "path_glups": SAMPLE_EVERY * V / (pms * 1e-3) / 1e9,
                             "sample_ms": max(pms - SAMPLE_EVERY * ms, 0.0),
                             "steps_per_launch": lf["steps_per_launch"],
                             "achieved_GBs": lf["achieved_GBs"],
                             "launch_shape": list(shape) + [list(h.time_blocking())]}
                h.close()
            cq = dict(workloads.CONFIGS[args.workload])
            h = flb.Lattice(cq["nx"], cq["ny"], cq["tau"], 0.0, rho0=cq["rho0"], u0=cq["u0"],
                            seed=cq["seed"], storage=args.storage)
            h.set_stream(stream)
            h.autotune(50)
            ms = steady_step_ms(torch, h, stream)
            forms["noise_off_" + args.storage] = {"step_glups": V / (ms * 1e-3) / 1e9}
            out["noise_overhead"] = iso_ms / ms - 1.0
            h.close()
            for name, specs in (("batched_gi_96x512", workloads.gi_sweep_specs()),
                                ("batched_uneven_64", workloads.uneven_batch_specs())):
                forms[name] = batched_form(torch, flb, stream, specs, args.storage)
                print(f"bench: {name} {forms[name]}", file=sys.stderr, flush=True)
            # one GPU's share of the 4096^2 lattice split into eight x-strips
            # (the halo and all-to-all exchanges are not built: the strip is
            # periodic here); its step rate, and its sample, whose row
            # transforms are the strip's own part of the distributed one
            forms["shard_512x4096"] = shard_form(torch, flb, workloads, stream, args.workload,
                                                 args.storage)
            print(f"bench: shard {forms['shard_512x4096']}", file=sys.stderr, flush=True)
            # the other velocity sets the paper tested (Sec. 3)
            forms["d3q15_256x256x256"] = velocity_set_form(torch, flb, stream, "D3Q15",
                                                           (256, 256, 256))
            forms["d1q3_67108864"] = velocity_set_form(torch, flb, stream, "D1Q3", (1 << 26,),
                                                       sample=False)
            print(f"bench: velocity sets {forms['d3q15_256x256x256']} {forms['d1q3_67108864']}",
                  file=sys.stderr, flush=True)
        out["forms"] = forms

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(workloads, args.workload)
    print(json.dumps(out), flush=True)
    g.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
