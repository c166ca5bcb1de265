#!/usr/bin/env python3
"""Benchmark of the batched Monte Carlo propagation hot path on one MI355X.

One bench step = one fsg_simulate call: seeds -> synchronous pull steps until
absorption or the step cap -> final states [n][B] and per-node counts, for a
batch of B replicates of the workload.  Inputs are resident in HBM before the
timed region.  The metric is replicate-edge updates per second:
nnz * B * steps_run / wall time of the step.

Workloads (synthetic stand-ins for the paper's datasets):
  c4  IC weighted cascade on R-MAT scale 26 (2^26 nodes, edge factor 16,
      2^30 arcs), 50 seeds, B=64, to absorption  (default: the largest
      single-GPU configuration, the web-scale run of Sec. 5)
  c2  SIR on Chung-Lu n=1e6 (exponent 2.5, mean degree 20), beta 0.02,
      gamma 0.1, 1% seeds, B=1024, 200 steps
  c1  IC on directed G(1000, mean out-degree 10), p 0.1, B=100
  c5  learned surrogate: GNN trained on simulator labels (Chung-Lu n=1e5,
      4 graphs x 500 seed sets x 1024 replicates), evaluated on 2 unseen
      graphs x 100 queries against 4096-replicate Monte Carlo
  c3  64 mixed jobs (Chung-Lu n log-uniform in [1e4, 2e6], mean degree
      U(5, 50); IC p=0.05 / SIR beta 0.03 gamma 0.1 / LT; B log-uniform in
      [64, 4096]; 1-1000 seeds) in one batched, graph-captured launch per step
  hk  Hegselmann-Krause opinion dynamics on the c2 graph, eps 0.32, B=256
      uniform [-1, 1] initial opinion vectors, 20 steps (FP32 state)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# Philox4x32-10 calls per second chip-wide: one call is 20 v_mad_u64_u32 (8
# cycles per wave64 on a SIMD) and 20 v_bitop3_b32 (4 cycles) in the build's
# ISA, 240 SIMD cycles per 64 calls; 1024 SIMDs (256 CUs x 4) at 2.4 GHz
PEAK_PHILOX_CALLS = 1024 * 2.4e9 * 64 / 240.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


# HIP sources each workload's dominant kernel is built and launched from
KERNEL_SOURCES = {
    "hk": ["fsg_hk.hip", "fsg_internal.hpp"],
    "c5": ["fsg_gnn.hip", "fsg_internal.hpp"],
}
SIM_SOURCES = ["fsg_kernels.hip", "fsg_device.hpp", "fsg_internal.hpp", "fsg_abi.hip"]


def strip_comments(src: str) -> str:
    """C/C++ source without its comments and with runs of whitespace made one
    space (string and character literals kept as written)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c == "/" and src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif c == "/" and src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash(workload: str = "c2") -> str:
    """Hash of the HIP sources behind a workload's kernels, comments and
    layout left out; a counter record is valid only for the hash it was
    taken at."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_14895_amd", "csrc")
    for name in sorted(KERNEL_SOURCES.get(workload, SIM_SOURCES)):
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update(name.encode() + b"\0" + strip_comments(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str = None):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter record (FETCH_SIZE and WRITE_SIZE, scaled by what the
    same counters read for a plain copy of known size), or None when the
    kernels changed since the record was taken or the record is of another
    kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_source_hash") != kernel_source_hash(workload):
        return None
    if kernel is not None and rec.get("kernel") != kernel:
        return None
    return rec.get("hbm_bytes_per_launch")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _finite(x):
    """NaN / infinity -> None, recursively, so the line stays valid JSON."""
    import math
    if isinstance(x, float) and not math.isfinite(x):
        return None
    if isinstance(x, dict):
        return {k: _finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_finite(v) for v in x]
    return x


def emit(out: dict):
    print(json.dumps(_finite(out), allow_nan=False), flush=True)


def algorithmic_bytes_per_step(model: str, n: int, nnz: int, B: int, edge_parallel: bool) -> float:
    """Bytes one pull step must move if every array is touched once per use.

    Row-group kernel: sources 4 B/arc, row pointers 4 B/row, the gathered
    neighbour word group 8 W B/arc, and the node's own planes (IC: read A,
    write A and F; SIR-family: read h, r, write h, r; LT: read and write the
    active plane).
    Edge-parallel IC kernel (B <= 64): sources 4 B/arc and one read of the
    N-bit frontier bitmap; the target rows, degrees and words of the few
    frontier arcs are not counted."""
    if edge_parallel:
        return 4.0 * nnz + n / 8.0
    W = (B + 63) // 64
    own = {"ic": 24, "lt": 16}.get(model, 32) * W
    return 4.0 * nnz + 8.0 * W * nnz + 4.0 * (n + 1) + own * n


def finalize_bytes(model: str, n: int, B: int, states: bool, bitmap: bool,
                   ever_nodes=None) -> float:
    """Bytes the finalize kernel must move: per node the packed words it
    reads (the state-1 plane, except where a frontier bitmap marks it empty;
    the removed / ever-active plane for IC, SIR, SEIR; the latent plane for
    SEIR, SEIS), the uint8 states it writes ([n][B], if asked) and the uint32
    count; plus one read of the n-bit frontier bitmap.  The frontier-driven
    IC run (ever_nodes = the nodes some replicate activated) reads and clears
    the ever-active word only of those nodes, and reads and clears the n-bit
    bitmap that lists them."""
    W = (B + 63) // 64
    if ever_nodes is not None:
        return n * ((B if states else 0) + 4.0) + 3 * n / 8.0 + 16.0 * W * ever_nodes
    planes = (0 if bitmap else 1) + (1 if model in ("ic", "sir", "seir") else 0) + \
        (1 if model in ("seir", "seis") else 0)
    return n * (8.0 * W * planes + (B if states else 0) + 4.0) + (n / 8.0 if bitmap else 0.0)


def make_workload(name: str):
    from paper_2603_14895_amd import workloads as Wl
    if name == "c1":
        return Wl.config_c1()
    if name == "c2":
        return Wl.config_c2()
    if name == "c4":
        dev = "cuda"
        return Wl.config_c4(device=dev)
    raise SystemExit(f"unknown workload {name}")


def params_of(c):
    if c["model"] == "ic":
        return dict(p=c.get("p", 0.0), ic_prob=c.get("ic_prob", "uniform"),
                    max_steps=c["max_steps"])
    if c["model"] in ("sir", "sis", "si"):
        return dict(beta=c["beta"], gamma=c["gamma"], max_steps=c["max_steps"])
    return dict(max_steps=c["max_steps"])


def host_cpu():
    """Host threads the oracle may use and what the host is: the CPUs this
    process may run on (sched_getaffinity), capped by OMP_NUM_THREADS when it
    is set (the host's CPU share per GPU), plus the CPU model name."""
    try:
        visible = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        visible = os.cpu_count() or 1
    threads = visible
    share = os.environ.get("OMP_NUM_THREADS", "")
    if share.isdigit() and int(share) > 0:
        threads = min(threads, int(share))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"threads": max(1, threads), "visible_cpus": visible, "omp_num_threads": share or None,
            "cpu_model": model}


def cpu_fields(hc):
    return {"cores": hc["threads"], "cpu_model": hc["cpu_model"],
            "visible_cpus": hc["visible_cpus"], "omp_num_threads": hc["omp_num_threads"]}


def cpu_baseline(c, ptr, src, target_seconds: float):
    """The oracle as it stands on a bounded sample of the same workload: a
    subset of the replicates (a multiple of the host thread count, sized to
    roughly `target_seconds`), same graph, seeds, key and step cap.  Rate in
    replicate-edge updates per second."""
    import oracle
    hc = host_cpu()
    threads = hc["threads"]
    okw = dict(params_of(c))
    if "ic_prob" in okw:
        from paper_2603_14895_amd import fsg
        okw["ic_prob"] = fsg.IC_PROBS[okw["ic_prob"]]

    def run(R):
        t0 = time.perf_counter()
        if c["model"] == "ic" and ptr.size > 50_000_000:
            # the plain loop nest is far too slow at web scale: the live-edge
            # BFS oracle computes the same final states
            _, _, _, steps, _ = oracle.ic_live_edge(ptr, src, c["seeds"], R, c["rng_key"],
                                                    want_states=False, nthreads=threads, **okw)
            kind = "oracle-live-edge-bfs"
        else:
            _, _, steps, _ = oracle.simulate(c["model"], ptr, src, c["seeds"], R, c["rng_key"],
                                             want_states=False, nthreads=threads, **okw)
            kind = "oracle"
        return time.perf_counter() - t0, steps, kind

    R = min(threads, c["B"])
    dt, steps, kind = run(R)
    if dt < target_seconds / 2 and R < c["B"] and kind == "oracle":
        R = min(c["B"], R * max(1, int(round(target_seconds / max(dt, 1e-3)))))
        dt, steps, kind = run(R)
    rate = src.size * R * steps / dt
    return {"value": rate, "unit": "replicate-edge updates/s", **cpu_fields(hc), "kind": kind,
            "sample": f"{R} replicates (of B={c['B']}) x {steps} steps on the full graph, "
                      f"{dt:.1f} s"}


def frontier_arcs(dg, c, outdeg):
    """Arcs whose source is in some replicate's frontier, per step of one IC
    run (outside the timed region): the run is repeated with the stepping
    interface, and after each step the nodes holding a newly active replicate
    are summed by out-degree.  These are the arcs the frontier-bitmap kernel
    must process; the rest of its source stream only confirms that a source
    is not in the frontier."""
    import numpy as np
    import torch

    from paper_2603_14895_amd import fsg
    sess = fsg.Session(dg, c["model"], c["seeds"], c["B"], c["rng_key"], **params_of(c))
    out = []
    try:
        seeds = torch.zeros(dg.n, dtype=torch.bool, device="cuda")
        seeds[torch.from_numpy(np.asarray(c["seeds"], dtype=np.int64)).to("cuda")] = True
        front = seeds
        while True:
            out.append(int(outdeg[front].sum().item()))
            info, _ = sess.step(1)
            st, _, _ = sess.read(want_states=True)
            front = (st == 1).any(dim=1)
            del st
            if int(info.absorbed) or not bool(front.any().item()):
                break
    finally:
        sess.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4", "c5", "hk"])
    ap.add_argument("--epochs", type=int, default=8, help="surrogate training epochs (c5)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the schedule(s) first with the library autotuner")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file")
    ap.add_argument("--steps-per-sync", type=int, default=0,
                    help="c3: batched steps per captured chunk (0: the binding's default)")
    ap.add_argument("--blocks-per-cu", type=int, default=0,
                    help="c3: persistent blocks of the batched kernels per CU (0: default)")
    ap.add_argument("--tune-trials", type=int, default=32,
                    help="c3: whole-batch trials of the batch autotuner")
    ap.add_argument("--tune-steps", type=int, default=0,
                    help="autotuner window: runs of K and 2K steps per candidate; 0 = the "
                         "workload's step cap (whole runs), or 64 for runs to absorption")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-frontier", action="store_true",
                    help="IC workloads: skip the per-step count of live frontier arcs")
    ap.add_argument("--no-out-adjacency", action="store_true",
                    help="do not bind the out-adjacency (IC with B <= 64: streaming step only; "
                         "no tail mode)")
    ap.add_argument("--stream-reference", type=int, default=5,
                    help="frontier-driven IC: also time this many runs of the streaming step")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--schedule", default=None, help="JSON dict of fsg_schedule fields")
    ap.add_argument("--no-states", action="store_true", help="counts only (no [n][B] output)")
    ap.add_argument("--print-kernel-hash", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.print_kernel_hash:
        print(json.dumps({w: kernel_source_hash(w) for w in ("c1", "c2", "c3", "c4", "c5", "hk")}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single GPU (replicates "
              "would shard across GPUs by global replicate index); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2603_14895_amd import fsg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        xa = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
        xb = torch.empty_like(xa)
        torch.cuda.synchronize()
        xb.copy_(xa)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {nb} bytes read + {nb} bytes written")
        del xa, xb
    if args.workload == "c3":
        return bench_batch(args)
    if args.workload == "c5":
        return bench_surrogate(args)
    if args.workload == "hk":
        return bench_hk(args)
    t0 = time.perf_counter()
    c = make_workload(args.workload)
    gr = c["graph"]
    ptr, src = gr.numpy()
    log(f"[bench] workload {c['name']}: n={gr.n} nnz={gr.nnz} B={c['B']} "
        f"(generated in {time.perf_counter() - t0:.1f}s)")
    del gr
    c["graph"] = None
    # the out-adjacency: the frontier-driven IC step (one word per node), and
    # the tail mode of the pull step (candidate rows from the out-arcs of the
    # infected or newly activated nodes)
    want_out = c["model"] in ("ic", "si", "sis", "sir", "lt") and not args.no_out_adjacency
    t_b = time.perf_counter()
    dg = fsg.DeviceGraph(ptr, src, device="cuda:0", out=want_out)
    log(f"[bench] graph bound{' with its out-adjacency' if want_out else ''} in "
        f"{time.perf_counter() - t_b:.1f}s")
    sched = json.loads(args.schedule) if args.schedule else {}
    if args.autotune:
        ts = args.tune_steps or (c["max_steps"] if c["max_steps"] > 0 else 64)
        tuned, bms, dms = fsg.autotune(dg, c["model"], c["seeds"], c["B"], c["rng_key"],
                                       tune_steps=ts, cache_path=args.tune_cache, **params_of(c))
        log(f"[bench] autotuned {tuned}: {bms:.4f} ms/step vs default {dms:.4f}")
        sched.update({k: v for k, v in tuned.items() if v})
    sched["time_kernels"] = 1
    sim = fsg.Simulation(dg, c["model"], c["B"], schedule=sched, want_states=not args.no_states,
                         **params_of(c))
    log(f"[bench] workspace {sim.ws_bytes / 2**30:.2f} GiB, schedule "
        f"{fsg.fsg_default_schedule(dg.handle, sim.prm, c['B']).as_dict()} overrides {sched}")
    # runs after the first reuse the object's private workspace (each run
    # still computes everything from the seeds)
    for i in range(args.warmup):
        info = sim.run(c["seeds"], c["rng_key"])
        log(f"[bench] warmup {i}: steps_run={info.steps_run} absorbed={info.absorbed}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total_updates = 0.0
    kernel_ms = fin_ms = setup_ms = 0.0
    launches = tail_launches = 0
    steps_seen = []
    for i in range(args.steps):
        info = sim.run(c["seeds"], c["rng_key"])
        total_updates += float(src.size) * c["B"] * info.steps_run
        kernel_ms += info.step_kernel_ms
        launches += info.step_launches
        tail_launches += info.tail_steps
        fin_ms += info.finalize_ms
        setup_ms += info.setup_ms
        steps_seen.append(int(info.steps_run))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    value = total_updates / dt
    ms_per_step = dt * 1000.0 / args.steps
    counts = sim.counts.cpu().numpy()
    attack = float(counts.sum()) / (ptr.size - 1) / c["B"]
    log(f"[bench] {args.steps} steps in {dt:.3f}s: {ms_per_step:.2f} ms/step, "
        f"steps_run={steps_seen}, mean counted fraction {attack:.4f}")

    used = fsg.fsg_default_schedule(dg.handle, sim.prm, c["B"]).as_dict()
    used.update({k: v for k, v in sched.items() if v})
    variant = used.get("kernel_variant")
    n = ptr.size - 1
    step_kernel = {3: "k_ic_front", 2: "k_ic_stream"}.get(variant, "k_step")
    avg_kernel_ms = kernel_ms / max(launches, 1)
    kernels = {step_kernel: {"avg_launch_ms": round(avg_kernel_ms, 5), "launches": launches,
                             "ms_per_run": round(kernel_ms / args.steps, 4)},
               "k_finalize": {"avg_launch_ms": round(fin_ms / args.steps, 5),
                              "launches": args.steps if fin_ms > 0 else 0,
                              "ms_per_run": round(fin_ms / args.steps, 4)},
               "setup": {"ms_per_run": round(setup_ms / args.steps, 4),
                         "note": "plane fills, table uploads and seeding, host gaps included"}}
    log(f"[bench] device time per run: {json.dumps(kernels)}")
    # the roofline of the kernel with the most device time per run
    if fin_ms > kernel_ms:
        ever = int((counts > 0).sum()) if variant == 3 else None
        abytes = finalize_bytes(c["model"], n, c["B"], not args.no_states, variant in (2, 3), ever)
        kname, avg_ms, nl = "k_finalize", fin_ms / args.steps, args.steps
    else:
        if variant == 3:
            # per live arc: its (target, edge id) entry, the target's
            # ever-active word and in-degree (24 bytes); the frontier nodes'
            # own words and work items are left out
            outdeg = torch.bincount(torch.from_numpy(src).to("cuda"), minlength=n)
            live = frontier_arcs(dg, c, outdeg)
            del outdeg
            abytes = 24.0 * float(sum(live)) / max(1, launches // args.steps)
        else:
            abytes = algorithmic_bytes_per_step(c["model"], n, src.size, c["B"], variant == 2)
            if tail_launches:
                # tail-mode steps (SI family) leave out the rows that cannot
                # change: counted here as moving nothing, so the mean over the
                # launches is a lower bound
                abytes *= (launches - tail_launches) / max(launches, 1)
        kname, avg_ms, nl = step_kernel, avg_kernel_ms, launches
    achieved = abytes / (avg_ms / 1e3) / 1e9
    traffic = measured_traffic(args.workload, kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic,
                "frac_measured": (round(traffic / (avg_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)
                                  if traffic else None),
                "kernel": kname, "avg_launch_ms": round(avg_ms, 5), "launches": nl,
                "algorithmic_bytes_per_launch": abytes,
                "tail_mode_launches": tail_launches}
    roofline_other = None
    if c["model"] in ("sir", "sis", "si", "seir", "seis") and kname == "k_step":
        # a counting run gives the generator calls per step: the arithmetic
        # ceiling of the same launches
        cnt_sim = fsg.Simulation(dg, c["model"], c["B"], want_states=False,
                                 schedule=dict(sched, time_kernels=0,
                                               options=fsg.OPT_COUNT_DRAWS), **params_of(c))
        ci = cnt_sim.run(c["seeds"], c["rng_key"])
        del cnt_sim
        calls = int(ci.philox_calls) / max(int(ci.steps_run), 1)
        rate = calls / (avg_kernel_ms / 1e3)
        alu = {"bound": "alu", "achieved": rate, "peak": PEAK_PHILOX_CALLS,
               "unit": "Philox4x32-10 calls/s", "frac": round(rate / PEAK_PHILOX_CALLS, 4),
               "traffic": None, "kernel": "k_step", "avg_launch_ms": round(avg_kernel_ms, 5),
               "launches": launches, "calls_per_launch": calls}
        hbm_meas = roofline["traffic"] / (avg_kernel_ms / 1e3) / 1e9 / PEAK_HBM_GBS \
            if roofline["traffic"] else None
        roofline["frac_measured"] = round(hbm_meas, 4) if hbm_meas is not None else None
        log(f"[bench] generator calls per step {calls:.4g}: {alu['frac']:.3f} of the ALU ceiling; "
            f"HBM {roofline['frac']:.3f} (algorithmic), {hbm_meas} (counters)")
        # the binding ceiling is the one the kernel comes closer to (HBM by
        # its measured traffic when the counter record is current)
        if alu["frac"] > (hbm_meas if hbm_meas is not None else roofline["frac"]):
            roofline, roofline_other = alu, roofline
        else:
            roofline_other = alu
    stream_ref = None
    if variant == 3 and args.stream_reference > 0:
        # the same runs with the streaming step (every arc read every step),
        # for comparison; not part of the value
        ref = fsg.Simulation(dg, c["model"], c["B"], want_states=not args.no_states,
                             schedule=dict(sched, kernel_variant=2), **params_of(c))
        ref.run(c["seeds"], c["rng_key"])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        km, kl = 0.0, 0
        for _ in range(args.stream_reference):
            ri = ref.run(c["seeds"], c["rng_key"])
            km += ri.step_kernel_ms
            kl += ri.step_launches
        torch.cuda.synchronize()
        d2 = time.perf_counter() - t2
        sb = algorithmic_bytes_per_step(c["model"], n, src.size, c["B"], True)
        stream_ref = {"kernel": "k_ic_stream", "ms_per_run": round(d2 * 1e3 / args.stream_reference, 3),
                      "value": float(src.size) * c["B"] * int(ri.steps_run) * args.stream_reference / d2,
                      "avg_launch_ms": round(km / max(kl, 1), 5),
                      "hbm_frac_algorithmic": round(sb / (km / max(kl, 1) / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
        log(f"[bench] streaming step for comparison: {stream_ref}")
        del ref
    frontier = None
    if c["model"] == "ic" and not args.no_frontier:
        outdeg = torch.bincount(torch.from_numpy(src).to("cuda"), minlength=ptr.size - 1)
        live = frontier_arcs(dg, c, outdeg)
        del outdeg
        frontier = {"live_arcs_per_step": live,
                    "live_arc_fraction_mean": round(float(np.mean(live)) / src.size, 6),
                    "note": "arcs out of nodes with a newly active replicate, per step: the "
                            "arcs the frontier-driven step pushes over; the streaming step "
                            "reads every source to find them"}
        log(f"[bench] live frontier arcs per step: {live}")
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(c, ptr, src, args.cpu_seconds)
        log(f"[bench] cpu baseline {cpu}")
    out = {
        "metric": "replicate-edge updates/s", "value": value, "unit": "replicate-edge updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64 bit-packed replicates / u32 integer draws",
        "data": "synthetic",
        "config": {"workload": c["name"], "model": c["model"], "n": int(ptr.size - 1),
                   "nnz": int(src.size), "B": c["B"], "max_steps": c["max_steps"],
                   "steps_run": steps_seen[-1] if steps_seen else 0, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "runs_per_s": round(args.steps / dt, 3),
        "kernels": kernels,
    }
    if frontier is not None:
        out["frontier"] = frontier
    if stream_ref is not None:
        out["streaming_step_reference"] = stream_ref
    if roofline_other is not None:
        out["roofline_other"] = roofline_other
    emit(out)


def hk_algorithmic_bytes(n: int, nnz: int, B: int) -> float:
    """Bytes one Hegselmann-Krause step must move: the B opinions of every
    arc's source (4 B each), the node's own opinions read and written, the
    sources (4 B/arc) and row pointers (4 B/row)."""
    return 4.0 * B * nnz + 8.0 * B * n + 4.0 * nnz + 4.0 * (n + 1)


def bench_hk(args):
    """Hegselmann-Krause opinion dynamics: one bench step = one fsg_hk call
    (reset to the initial opinions, then up to max_steps synchronous steps)."""
    import numpy as np
    import torch

    from paper_2603_14895_amd import fsg
    from paper_2603_14895_amd import workloads as Wl

    t0 = time.perf_counter()
    c = Wl.config_hk()
    ptr, src = c["graph"].numpy()
    n, B, K, eps = ptr.size - 1, c["B"], c["max_steps"], c["eps"]
    h0 = Wl.uniform_opinions(n, B, c["opinion_seed"])
    log(f"[bench] workload {c['name']}: n={n} nnz={src.size} B={B} "
        f"(generated in {time.perf_counter() - t0:.1f}s)")
    c["graph"] = None
    dg = fsg.DeviceGraph(ptr, src, device="cuda:0")
    sched = json.loads(args.schedule) if args.schedule else {}
    sched["time_kernels"] = 1
    sc = fsg.make_schedule(sched)
    h0d = torch.from_numpy(h0).to("cuda:0")
    h = torch.empty_like(h0d)
    counts = torch.empty(B, dtype=torch.int32, device="cuda:0")
    nb = fsg.fsg_hk_workspace_size(dg.handle, B, sc)
    ws, addr = fsg._ws(nb, "cuda:0")

    def one():
        h.copy_(h0d)
        return fsg.fsg_hk(dg.handle, eps, K, B, h.data_ptr(), sc, addr, nb, 0.5, counts.data_ptr())

    for i in range(args.warmup):
        info = one()
        log(f"[bench] warmup {i}: steps_run={info.steps_run} converged={info.absorbed}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    updates, kernel_ms, launches, steps_seen = 0.0, 0.0, 0, []
    for i in range(args.steps):
        info = one()
        updates += float(src.size) * B * info.steps_run
        kernel_ms += info.step_kernel_ms
        launches += info.step_launches
        steps_seen.append(int(info.steps_run))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    value = updates / dt
    ms_per_step = dt * 1000.0 / args.steps
    above = float(counts.sum().item()) / n / B
    log(f"[bench] {args.steps} steps in {dt:.3f}s: {ms_per_step:.2f} ms/step, steps_run={steps_seen}, "
        f"mean fraction of opinions above 0.5: {above:.4f}")
    avg_kernel_ms = kernel_ms / max(launches, 1)
    abytes = hk_algorithmic_bytes(n, src.size, B)
    achieved = abytes / (avg_kernel_ms / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": measured_traffic("hk"), "kernel": "k_hk_step",
                "avg_launch_ms": round(avg_kernel_ms, 5), "launches": launches,
                "algorithmic_bytes_per_launch": abytes}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        hc = host_cpu()
        threads = hc["threads"]
        R, S = threads, 2
        hs = np.ascontiguousarray(h0[:, :R])
        t2 = time.perf_counter()
        _, st, _ = oracle.hk(ptr, src, hs, eps, S, nthreads=threads)
        dc = time.perf_counter() - t2
        if dc < args.cpu_seconds / 2:
            S = max(S, min(K, int(S * args.cpu_seconds / max(dc, 1e-3))))
            t2 = time.perf_counter()
            _, st, _ = oracle.hk(ptr, src, hs, eps, S, nthreads=threads)
            dc = time.perf_counter() - t2
        cpu = {"value": src.size * R * st / dc, "unit": "replicate-edge updates/s",
               **cpu_fields(hc), "kind": "oracle",
               "sample": f"{R} replicates (of B={B}) x {st} steps on the full graph, {dc:.1f} s"}
        log(f"[bench] cpu baseline {cpu}")
    del ws
    out = {
        "metric": "replicate-edge updates/s", "value": value, "unit": "replicate-edge updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": c["name"], "model": "hk", "n": int(n), "nnz": int(src.size), "B": B,
                   "eps": eps, "max_steps": K, "steps_run": steps_seen[-1] if steps_seen else 0,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    emit(out)


def bench_batch(args):
    """The mixed batched workload: one fsg_batch_run over all jobs per step."""
    import numpy as np
    import torch

    from paper_2603_14895_amd import fsg
    from paper_2603_14895_amd import workloads as Wl

    t0 = time.perf_counter()
    specs = Wl.config_c3_jobs()
    jobs, host = [], []
    for sp in specs:
        gr = Wl.build_c3_graph(sp, device="cuda")
        ptr, src = gr.numpy()
        del gr
        # every job binds the out-adjacency: the tail mode marks candidate rows
        # from the out-arcs of the nodes that changed
        dg = fsg.DeviceGraph(ptr, src, device="cuda:0", out=not args.no_out_adjacency)
        seeds = Wl.uniform_seeds(dg.n, sp["n_seeds"], sp["seed_seed"])
        prm = {k: sp[k] for k in ("p", "ic_prob", "beta", "gamma", "max_steps") if k in sp}
        jobs.append(dict(graph=dg, model=sp["model"], B=sp["B"], seeds=seeds, rng_key=sp["key"],
                         **prm))
        host.append((ptr, src))
    tot_nnz = sum(h[1].size for h in host)
    log(f"[bench] c3: {len(jobs)} jobs, {tot_nnz} arcs, B mean "
        f"{np.mean([j['B'] for j in jobs]):.0f} (built in {time.perf_counter() - t0:.1f}s)")
    batch = fsg.Batch(jobs, steps_per_sync=args.steps_per_sync or fsg.BATCH_STEPS_PER_SYNC,
                      want_states=not args.no_states,
                      blocks_per_cu=args.blocks_per_cu or None)
    tune = None
    if args.autotune:
        # the batch is tuned as a batch: whole runs scored by device time
        t1 = time.perf_counter()
        tune = batch.autotune(max_trials=args.tune_trials)
        by_model = {}
        for j, sc in zip(jobs, tune["schedules"]):
            key = {k: sc.get(k, 0) for k in ("row_lanes", "tile_edges", "heavy_threshold")}
            by_model.setdefault(j["model"], [])
            if key not in by_model[j["model"]]:
                by_model[j["model"]].append(key)
        tune["schedules_by_model"] = by_model
        log(f"[bench] batch autotune: {tune['default_ms']:.1f} -> {tune['best_ms']:.1f} ms device "
            f"in {tune['trials']} trials ({time.perf_counter() - t1:.1f}s); steps_per_sync "
            f"{tune['steps_per_sync']}, blocks per CU {tune['blocks_per_cu']}; schedules {by_model}")
    log(f"[bench] batch workspace {batch.ws_bytes / 2**30:.2f} GiB")
    for i in range(args.warmup):
        infos, ms = batch.run()
        log(f"[bench] warmup {i}: {ms:.1f} ms device, steps {[int(x.steps_run) for x in infos]}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total_updates, dev_ms = 0.0, 0.0
    for _ in range(args.steps):
        infos, ms = batch.run()
        dev_ms += ms
        total_updates += sum(float(h[1].size) * j["B"] * x.steps_run
                             for h, j, x in zip(host, jobs, infos))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    steps_run = [int(x.steps_run) for x in infos]
    # every word of a job counted at each of its dense steps; steps in the
    # tail mode leave out the rows that cannot change and count as nothing
    abytes = sum(algorithmic_bytes_per_step(j["model"], h[0].size - 1, h[1].size, j["B"], False)
                 * (x.steps_run - x.tail_steps) for h, j, x in zip(host, jobs, infos))
    achieved = abytes * args.steps / (dev_ms / 1e3) / 1e9
    log(f"[bench] {args.steps} batch runs in {dt:.3f}s ({dev_ms / args.steps:.1f} ms device each); "
        f"tail-mode steps {sum(int(x.tail_steps) for x in infos)} of {sum(steps_run)}")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_batch(specs, jobs, host, args.cpu_seconds)
        log(f"[bench] cpu baseline {cpu}")
    out = {
        "metric": "replicate-edge updates/s", "value": total_updates / dt,
        "unit": "replicate-edge updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1000.0 / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64 bit-packed replicates / u32 integer draws", "data": "synthetic",
        "tail_mode_steps": [int(x.tail_steps) for x in infos],
        "config": {"workload": "c3_mixed_batch_64_jobs", "jobs": len(jobs), "nnz_total": int(tot_nnz),
                   "B": [j["B"] for j in jobs], "steps_run": steps_run,
                   "autotuned": bool(args.autotune), "parallelism": "single GPU"},
        "autotune": ({k: tune[k] for k in ("default_ms", "best_ms", "trials", "steps_per_sync",
                                           "blocks_per_cu", "schedules_by_model")}
                     if tune else None),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic("c3"),
                     "frac_measured": (round(measured_traffic("c3") / (dev_ms / args.steps /
                                                                      max(1, max(steps_run)) / 1e3)
                                             / 1e9 / PEAK_HBM_GBS, 4)
                                       if measured_traffic("c3") else None),
                     "kernel": "k_batch_step + k_batch_combine (captured step chunks)",
                     "avg_launch_ms": round(dev_ms / args.steps / max(1, max(steps_run)), 5),
                     "launches": args.steps * max(steps_run),
                     "algorithmic_bytes_per_launch": abytes / max(1, max(steps_run))},
        "cpu_baseline": cpu,
    }
    emit(out)


def bench_surrogate(args):
    """The learned surrogate end to end: labels, training, threshold,
    evaluation against 4096-replicate Monte Carlo, timing of both."""
    import numpy as np
    import torch

    from paper_2603_14895_amd import fsg
    from paper_2603_14895_amd import surrogate as S
    from paper_2603_14895_amd import workloads as Wl

    n, gamma, K, B_lab, B_ref = 100_000, 0.1, 200, 1024, 4096
    rng = np.random.default_rng(Wl.BASE_SEED + 5)
    t0 = time.perf_counter()
    data, lab_ms, train_sets = [], 0.0, []
    for gi in range(4):
        gr = Wl.chung_lu(n, 20.0, 2.5, Wl.BASE_SEED + 50 + gi, device="cuda")
        ptr, src = gr.numpy()
        g = fsg.DeviceGraph(ptr, src)
        rv = fsg.DeviceGraph(*Wl.reverse_graph(gr).numpy())
        sets = S.seed_sets(n, 500, rng)
        betas = rng.uniform(0.01, 0.05, size=len(sets))
        y, sp, ms = S.mc_frequencies(g, sets, betas, gamma, K, B_lab, 1_000_000 * (gi + 1))
        lab_ms += ms
        data.append((g, rv, S.masks_of(sets, n), list(betas), y))
        train_sets.append(sets)
        log(f"[bench] labels graph {gi}: 500 seed sets x {B_lab} replicates in {ms:.0f} ms device, "
            f"mean spread {sp.mean() / n:.3f} n")
    ens = S.Ensemble(4, seed=Wl.BASE_SEED % 1000)
    t1 = time.perf_counter()
    ens.train(data, epochs=args.epochs, sets_per_step=8, lr=3e-3, progress_every=1)
    train_s = time.perf_counter() - t1
    # spread calibration fitted on the training queries' simulator labels
    tr_pred, tr_lab, tr_beta, tr_k = [], [], [], []
    for (g, rv, masks, betas, y), sets in zip(data, train_sets):
        tr_pred.append(ens.predict_spreads(g, masks, np.array(betas)).mean(axis=0))
        tr_lab.append(y.sum(dim=1).double().cpu().numpy())
        tr_beta += list(betas)
        tr_k += [len(x) for x in sets]
    coef = S.fit_calibration(np.concatenate(tr_pred), np.concatenate(tr_lab), tr_beta, tr_k)
    # held-out graphs: the gate is calibrated on the first 50 queries of each,
    # the rest are the test queries
    cal_s, cal_u, cal_r, cal_k, tests = [], [], [], [], []
    raw_err, calib_err = [], []  # every held-out query (calibration and test halves)
    ref_ms = 0.0
    for gi in range(2):
        gr = Wl.chung_lu(n, 20.0, 2.5, Wl.BASE_SEED + 90 + gi, device="cuda")
        g = fsg.DeviceGraph(*gr.numpy())
        qs = S.seed_sets(n, 100, rng)
        qb = rng.uniform(0.01, 0.05, size=len(qs))
        qk = np.array([len(np.unique(x)) for x in qs])
        _, ref, ms = S.mc_frequencies(g, qs, qb, gamma, K, B_ref, 7_000_000 * (gi + 1))
        ref_ms += ms
        mean, unc = S.uncertainty(ens.predict_spreads(g, S.masks_of(qs, n), qb))
        cal = S.apply_calibration(mean, qb, qk, coef)
        raw_err += list(np.abs(mean - ref) / ref)
        calib_err += list(np.abs(cal - ref) / ref)
        cal_s += list(cal[:50]); cal_u += list(unc[:50]); cal_r += list(ref[:50])
        cal_k += list(qk[:50])
        tests.append((g, qs[50:], qb[50:], ref[50:]))
        log(f"[bench] held-out graph {gi}: reference 100 x {B_ref} in {ms:.0f} ms device; "
            f"median error raw {np.median(np.abs(mean - ref) / ref):.4f}, "
            f"calibrated {np.median(np.abs(cal - ref) / ref):.4f}")
    gate = S.calibrate_gate(cal_s, cal_u, cal_r, cal_k, 0.02)
    gate["calib"] = list(coef)
    tau = gate["tau"]
    acc_err, fb_err, t_sur, n_fb, accepted = [], [], [], 0, []
    for g, qs, qb, ref in tests:
        est = fsg.SpreadEstimator(ens.members, g, gamma=gamma, max_steps=K, B_fallback=1024,
                                  gate=gate)
        for i in range(len(qs)):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            sp, u, fb = est.estimate(qs[i], qb[i], 31337 + i)
            dt = time.perf_counter() - ta
            (fb_err if fb else acc_err).append(abs(sp - ref[i]) / ref[i])
            n_fb += int(fb)
            if not fb:
                t_sur.append(dt)
                accepted.append((g, qs[i], qb[i], ref[i]))
    # plain Monte Carlo on the same GPU and the same accepted queries: 4096
    # replicates (the reference's cost) and the smallest B whose mean error
    # matches the surrogate's
    def mc_cost(B, count=20):
        errs, times = [], []
        for i, (g, q, b, r) in enumerate(accepted[:count]):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, cnt, _, _ = fsg.simulate(g, "sir", q, B, 4242 + i, beta=b, gamma=gamma,
                                        max_steps=K, want_states=False)
            s = float(cnt.sum().item()) / B
            times.append(time.perf_counter() - ta)
            errs.append(abs(s - r) / r)
        return float(np.mean(errs)), float(np.median(times))
    e_sur = float(np.mean(acc_err)) if acc_err else float("nan")
    t_s = float(np.median(t_sur)) if t_sur else float("nan")
    e4096, t4096 = mc_cost(B_ref) if accepted else (float("nan"), float("nan"))
    matched = None
    for B in (16, 32, 64, 128, 256, 512, 1024, 2048, 4096):
        if not accepted:
            break
        e, t = mc_cost(B)
        if e <= e_sur:
            matched = (B, e, t)
            break
    out = {
        "metric": "surrogate speed-up over 4096-replicate MC on accepted queries (spread err <= 2%)",
        "value": t4096 / t_s if t_sur else None, "unit": "x",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(t_s * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 weights/activations, fp32 accumulate (MFMA)", "data": "synthetic",
        "config": {"workload": "c5_surrogate_chunglu1e5", "n": n, "train_sets": 2000,
                   "label_replicates": B_lab, "reference_replicates": B_ref, "epochs": args.epochs,
                   "ensemble": 4, "tau": tau, "min_seeds": gate["min_seeds"],
                   "calibration": [round(float(c), 6) for c in coef], "parallelism": "single GPU"},
        "surrogate": {"accepted": len(acc_err), "fallback": n_fb, "acceptance": len(acc_err) / 100.0,
                      "heldout_raw_rel_err_median": float(np.median(raw_err)),
                      "heldout_raw_rel_err_p90": float(np.quantile(raw_err, 0.9)),
                      "heldout_calibrated_rel_err_median": float(np.median(calib_err)),
                      "heldout_calibrated_rel_err_p90": float(np.quantile(calib_err, 0.9)),
                      "heldout_queries": len(raw_err),
                      "accepted_rel_err_mean": e_sur,
                      "accepted_rel_err_max": float(np.max(acc_err)) if acc_err else None,
                      "fallback_rel_err_mean": float(np.mean(fb_err)) if fb_err else None,
                      "ms_per_query": t_s * 1e3, "mc4096_ms_per_query": t4096 * 1e3,
                      "mc4096_rel_err_mean": e4096,
                      "matched_accuracy_mc": ({"B": matched[0], "rel_err": matched[1],
                                               "ms_per_query": matched[2] * 1e3,
                                               "speedup": matched[2] / t_s} if matched else None),
                      "label_device_ms": lab_ms, "train_seconds": train_s,
                      "reference_device_ms": ref_ms},
        "roofline": None, "cpu_baseline": None,
    }
    log(f"[bench] c5 done in {time.perf_counter() - t0:.1f}s")
    emit(out)


def cpu_baseline_batch(specs, jobs, host, target_seconds):
    """The oracle on a bounded sample of the batch: the jobs in turn, each
    with as many replicates as the oracle has threads (it runs replicates in
    parallel, so every thread has one), until about target_seconds have
    passed."""
    import oracle
    hc = host_cpu()
    threads = hc["threads"]
    t0 = time.perf_counter()
    work, used = 0.0, 0
    for (ptr, src), j in zip(host, jobs):
        prm = {k: j[k] for k in ("p", "beta", "gamma", "max_steps") if k in j}
        if "ic_prob" in j:
            from paper_2603_14895_amd import fsg
            prm["ic_prob"] = fsg.IC_PROBS[j["ic_prob"]]
        R = min(threads, j["B"])
        _, _, steps, _ = oracle.simulate(j["model"], ptr, src, j["seeds"], R, j["rng_key"],
                                         want_states=False, nthreads=threads, **prm)
        work += float(src.size) * R * steps
        used += 1
        if time.perf_counter() - t0 > target_seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": work / dt, "unit": "replicate-edge updates/s", **cpu_fields(hc),
            "kind": "oracle",
            "sample": f"min({threads}, B) replicates of each of the first {used} jobs, {dt:.1f} s"}


if __name__ == "__main__":
    main()
