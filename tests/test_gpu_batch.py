"""Batched launch and autotuner on the GPU: every job of a mixed batch gives
the same bits as its solo run and as the oracle; tuned schedules change no
result."""
import os
import tempfile

import numpy as np
import pytest

from paper_2603_14895_amd import workloads as W
from tests.gpu_util import assert_same, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _params(j):
    return {k: j[k] for k in ("p", "ic_prob", "beta", "gamma", "alpha", "max_steps", "edge_p")
            if k in j}


def _mixed_jobs():
    rng = np.random.default_rng(11)
    specs = [
        ("ic", 2000, 8.0, 64, 0, dict(p=0.15, max_steps=-1), None),
        ("sir", 3000, 12.0, 1024, 0, dict(beta=0.04, gamma=0.1, max_steps=30), None),
        ("lt", 2500, 10.0, 100, 3, dict(max_steps=-1), None),
        ("sis", 1500, 6.0, 63, 1, dict(beta=0.1, gamma=0.2, max_steps=25), None),
        ("si", 1800, 5.0, 130, 0, dict(beta=0.05, max_steps=12), None),
        ("ic", 4000, 15.0, 300, 7, dict(p=0.05, ic_prob="weighted_cascade", max_steps=-1),
         dict(heavy_threshold=16, tile_edges=500)),
        ("sir", 2200, 20.0, 200, 0, dict(beta=0.02, gamma=0.3, max_steps=40),
         dict(row_lanes=4, heavy_threshold=30)),
        ("lt", 3000, 18.0, 1, 0, dict(max_steps=-1), dict(heavy_threshold=12)),
        ("ic", 1000, 10.0, 5, 0, dict(p=0.1, max_steps=2), None),
        ("sir", 800, 8.0, 64, 0, dict(beta=0.3, gamma=0.3, max_steps=0), None),
        ("seir", 2400, 14.0, 700, 0, dict(beta=0.04, alpha=0.3, gamma=0.1, max_steps=35), None),
        ("seis", 1700, 9.0, 90, 1, dict(beta=0.08, alpha=0.4, gamma=0.25, max_steps=20),
         dict(heavy_threshold=25)),
        # more than 16 words per node: words that stopped changing are left out
        ("lt", 1600, 12.0, 1100, 0, dict(max_steps=-1), dict(heavy_threshold=20)),
        ("ic", 1500, 10.0, 1500, 2, dict(p=0.1, max_steps=-1), None),
        ("sir", 1200, 10.0, 1300, 0, dict(beta=0.05, gamma=0.2, max_steps=40),
         dict(row_lanes=16, heavy_threshold=24)),
        ("swir", 2000, 10.0, 500, 2, dict(beta=0.1, alpha=0.1, gamma=0.4, max_steps=-1), None),
        ("swir", 1400, 16.0, 1090, 0, dict(beta=0.06, alpha=0.2, gamma=0.5, max_steps=-1),
         dict(heavy_threshold=18)),
    ]
    jobs = []
    for i, (model, n, deg, B, off, prm, sched) in enumerate(specs):
        gr = W.chung_lu(n, deg, 2.5, 700 + i)
        k = int(rng.integers(1, 30))
        seeds = W.uniform_seeds(gr.n, k, 800 + i) if i != 3 else np.array([], dtype=np.int32)
        jobs.append(dict(gr=gr, model=model, B=B, replicate_offset=off, seeds=seeds,
                         rng_key=0xBA7C0000 + i, schedule=sched, **prm))
    return jobs


def test_batch_equals_solo_and_oracle():
    from paper_2603_14895_amd import fsg
    jobs = _mixed_jobs()
    dgs = [fsg.DeviceGraph(*j["gr"].numpy()) for j in jobs]
    bj = [dict(graph=dg, **{k: v for k, v in j.items() if k != "gr"}) for dg, j in zip(dgs, jobs)]
    for spsync in (5, 16):
        batch = fsg.Batch(bj, steps_per_sync=spsync)
        infos, total_ms = batch.run()
        log(f"[batch] {len(jobs)} jobs, sync {spsync}: {total_ms:.2f} ms, "
            f"steps {[int(x.steps_run) for x in infos]}")
        for i, j in enumerate(jobs):
            got = (batch.states[i].cpu().numpy(), batch.counts[i].cpu().numpy().astype(np.uint32),
                   int(infos[i].steps_run), int(infos[i].absorbed))
            gnp = j["gr"].numpy()
            solo = gpu_run(gnp, j["model"], j["seeds"], j["B"], j["rng_key"],
                           replicate_offset=j["replicate_offset"], schedule=j["schedule"],
                           **_params(j))
            assert_same(got, solo, f"job {i} batched vs solo")
            ref = oracle_run(gnp, j["model"], j["seeds"], j["B"], j["rng_key"],
                             replicate_offset=j["replicate_offset"], **_params(j))
            assert_same(got, ref, f"job {i} batched vs oracle")
        batch.close()


def test_batch_tail_mode():
    """The tail mode in the batched launch: the mixed jobs on graphs with
    their out-adjacency bound, the mode forced on from the second chunk for
    every job (IC, SI, SIS, SIR, LT), then left to the library's per-job
    switch; every job equals the oracle, with chunks of 3 and 16."""
    from paper_2603_14895_amd import fsg
    jobs = _mixed_jobs()
    dgs = [fsg.DeviceGraph(*j["gr"].numpy(), out=True) for j in jobs]
    for forced, spsync in ((True, 3), (True, 16), (False, 3)):
        bj = []
        for dg, j in zip(dgs, jobs):
            d = dict(graph=dg, **{k: v for k, v in j.items() if k != "gr"})
            if forced:
                d["schedule"] = dict(j["schedule"] or {}, options=fsg.OPT_TAIL_ALWAYS)
            bj.append(d)
        batch = fsg.Batch(bj, steps_per_sync=spsync)
        infos, total_ms = batch.run()
        log(f"[batch] tail forced={forced} sync {spsync}: {total_ms:.2f} ms, tail steps "
            f"{[int(x.tail_steps) for x in infos]}")
        if forced:
            assert any(int(x.tail_steps) > 0 for x in infos)
        for i, j in enumerate(jobs):
            got = (batch.states[i].cpu().numpy(), batch.counts[i].cpu().numpy().astype(np.uint32),
                   int(infos[i].steps_run), int(infos[i].absorbed))
            ref = oracle_run(j["gr"].numpy(), j["model"], j["seeds"], j["B"], j["rng_key"],
                             replicate_offset=j["replicate_offset"], **_params(j))
            assert_same(got, ref, f"tail job {i} ({j['model']}) forced={forced} sync={spsync}")
        batch.close()


def test_batch_tail_mode_wide_rows():
    """The batched tail mode with rows of more than 64 words (B = 4200): the
    batched count reads such a row with a whole wave.  SIR and IC jobs beside
    a narrow LT job, the mode forced on and left to its switch; every job
    equals the oracle."""
    from paper_2603_14895_amd import fsg
    specs = [("sir", 900, 8.0, 4200, dict(beta=0.08, gamma=0.2, max_steps=40)),
             ("ic", 1100, 7.0, 4200, dict(p=0.1, max_steps=-1)),
             ("lt", 700, 6.0, 100, dict(max_steps=-1))]
    jobs = []
    for i, (model, n, deg, B, prm) in enumerate(specs):
        gr = W.chung_lu(n, deg, 2.5, 2301 + i)
        jobs.append(dict(gr=gr, model=model, B=B, seeds=W.uniform_seeds(n, 12, 2311 + i),
                         rng_key=0x7C00 + i, replicate_offset=0, **prm))
    dgs = [fsg.DeviceGraph(*j["gr"].numpy(), out=True) for j in jobs]
    for forced in (True, False):
        bj = []
        for dg, j in zip(dgs, jobs):
            d = dict(graph=dg, **{k: v for k, v in j.items() if k != "gr"})
            d["schedule"] = dict(options=fsg.OPT_TAIL_ALWAYS) if forced else None
            bj.append(d)
        batch = fsg.Batch(bj, steps_per_sync=3)
        infos, _ = batch.run()
        for i, j in enumerate(jobs):
            got = (batch.states[i].cpu().numpy(), batch.counts[i].cpu().numpy().astype(np.uint32),
                   int(infos[i].steps_run), int(infos[i].absorbed))
            prm = {k: j[k] for k in ("p", "beta", "gamma", "max_steps") if k in j}
            ref = oracle_run(j["gr"].numpy(), j["model"], j["seeds"], j["B"], j["rng_key"], **prm)
            assert_same(got, ref, f"wide tail job {i} ({j['model']}) forced={forced}")
        batch.close()


def test_batch_mixed_workload_small():
    """A reduced instance of the mixed batched workload (log-uniform sizes,
    B and seed-set sizes; IC / SIR / LT), every job checked on sampled
    replicates against the oracle and in full against its solo run."""
    from paper_2603_14895_amd import fsg
    specs = W.config_c3_jobs(n_jobs=9, n_hi=3e4, b_hi=700, seed_hi=100)
    dgs, bj, grs = [], [], []
    for sp in specs:
        gr = W.build_c3_graph(sp)
        grs.append(gr)
        dg = fsg.DeviceGraph(*gr.numpy())
        dgs.append(dg)
        seeds = W.uniform_seeds(gr.n, sp["n_seeds"], sp["seed_seed"])
        prm = {k: sp[k] for k in ("p", "ic_prob", "beta", "gamma", "max_steps") if k in sp}
        bj.append(dict(graph=dg, model=sp["model"], B=sp["B"], seeds=seeds, rng_key=sp["key"], **prm))
    batch = fsg.Batch(bj, steps_per_sync=16)
    infos, total_ms = batch.run()
    log(f"[batch] c3-small: {total_ms:.2f} ms")
    for i, (gr, j) in enumerate(zip(grs, bj)):
        gnp = gr.numpy()
        prm = {k: j[k] for k in ("p", "ic_prob", "beta", "gamma", "max_steps") if k in j}
        st = batch.states[i].cpu().numpy()
        solo = gpu_run(gnp, j["model"], j["seeds"], j["B"], j["rng_key"], **prm)
        got = (st, batch.counts[i].cpu().numpy().astype(np.uint32), int(infos[i].steps_run),
               int(infos[i].absorbed))
        assert_same(got, solo, f"c3-small job {i}")
        r0 = j["B"] // 3
        rs, _, _, _ = oracle_run(gnp, j["model"], j["seeds"], 2, j["rng_key"], replicate_offset=r0,
                                 **prm)
        assert (st[:, r0:r0 + 2] == rs).all(), i
    batch.close()


def test_batch_autotune_tuned_batch_matches_oracle():
    """The batch autotuner times whole batch runs over its search space and
    never returns a configuration slower than the one it started from; the
    batch re-planned with the tuned schedules and launch gives every job's
    oracle bits (sampled replicates) and its solo run's bits."""
    from paper_2603_14895_amd import fsg
    specs = W.config_c3_jobs(n_jobs=7, n_hi=2e4, b_hi=600, seed_hi=80, seed=4242)
    dgs, bj, grs = [], [], []
    for sp in specs:
        gr = W.build_c3_graph(sp)
        grs.append(gr)
        dg = fsg.DeviceGraph(*gr.numpy())
        dgs.append(dg)
        seeds = W.uniform_seeds(gr.n, sp["n_seeds"], sp["seed_seed"])
        prm = {k: sp[k] for k in ("p", "ic_prob", "beta", "gamma", "max_steps") if k in sp}
        bj.append(dict(graph=dg, model=sp["model"], B=sp["B"], seeds=seeds, rng_key=sp["key"], **prm))
    batch = fsg.Batch(bj, steps_per_sync=16)
    res = batch.autotune(max_trials=14)
    log(f"[batch] autotune: {res['default_ms']:.2f} -> {res['best_ms']:.2f} ms in {res['trials']} "
        f"trials, sync {res['steps_per_sync']}, blocks/CU {res['blocks_per_cu']}")
    assert res["best_ms"] <= res["default_ms"] + 1e-9 and 1 <= res["trials"] <= 14
    infos, _ = batch.run()
    for i, (gr, j) in enumerate(zip(grs, bj)):
        gnp = gr.numpy()
        prm = {k: j[k] for k in ("p", "ic_prob", "beta", "gamma", "max_steps") if k in j}
        st = batch.states[i].cpu().numpy()
        got = (st, batch.counts[i].cpu().numpy().astype(np.uint32), int(infos[i].steps_run),
               int(infos[i].absorbed))
        assert_same(got, gpu_run(gnp, j["model"], j["seeds"], j["B"], j["rng_key"], **prm),
                    f"tuned batch job {i} vs solo")
        r0 = j["B"] // 2
        rs, _, _, _ = oracle_run(gnp, j["model"], j["seeds"], 2, j["rng_key"], replicate_offset=r0,
                                 **prm)
        assert (st[:, r0:r0 + 2] == rs).all(), i
    batch.close()


def test_autotune_and_cache():
    from paper_2603_14895_amd import fsg
    gr = W.chung_lu(20000, 20.0, 2.5, 901)
    gnp = gr.numpy()
    dg = fsg.DeviceGraph(*gnp)
    seeds = W.uniform_seeds(gr.n, 200, 902)
    kw = dict(beta=0.03, gamma=0.1, max_steps=30)
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune.txt")
        best, bms, dms = fsg.autotune(dg, "sir", seeds, 512, 77, tune_steps=6, cache_path=cache, **kw)
        log(f"[tune] best {best} {bms:.4f} ms vs default {dms:.4f} ms")
        assert bms <= dms + 1e-9 and best["row_lanes"] >= 1
        again, bms2, dms2 = fsg.autotune(dg, "sir", seeds, 512, 77, tune_steps=6, cache_path=cache, **kw)
        assert again == best and dms2 < 0  # served from the cache
        tuned = gpu_run(gnp, "sir", seeds, 512, 0x77, schedule=best, **kw)
        plain = gpu_run(gnp, "sir", seeds, 512, 0x77, **kw)
        assert_same(tuned, plain, "tuned vs default schedule")
        assert_same(tuned, oracle_run(gnp, "sir", seeds, 512, 0x77, **kw), "tuned vs oracle")
        bb, _, _ = fsg.autotune(dg, "ic", seeds, 64, 5, tune_steps=4, batch_only=True, p=0.05)
        assert bb["kernel_variant"] == 1
        # windows longer than the poll interval cap (whole runs; the default window)
        for ts in (200, None):
            w, wms, dms3 = fsg.autotune(dg, "sir", seeds, 100, 78, tune_steps=ts, **kw)
            assert wms <= dms3 + 1e-9 and wms > 0
        w, _, _ = fsg.autotune(dg, "lt", seeds, 130, 79, tune_steps=100, max_steps=-1)
        assert w["row_lanes"] >= 1


def test_c3_full_size_every_job():
    """The mixed batched workload at full size (64 jobs, 3.4e8 arcs) in the
    launch configuration the benchmark times (every graph with its
    out-adjacency, so the jobs switch to the tail mode when few nodes change):
    every job equals its solo run bit for bit (compared on the device), and
    two sampled replicates of every job equal the oracle."""
    import torch
    from paper_2603_14895_amd import fsg
    specs = W.config_c3_jobs()
    jobs, host = [], []
    for sp in specs:
        gr = W.build_c3_graph(sp, device="cuda")
        ptr, src = gr.numpy()
        del gr
        dg = fsg.DeviceGraph(ptr, src, device="cuda:0", out=True)
        seeds = W.uniform_seeds(dg.n, sp["n_seeds"], sp["seed_seed"])
        prm = {k: sp[k] for k in ("p", "ic_prob", "beta", "gamma", "max_steps") if k in sp}
        jobs.append(dict(graph=dg, model=sp["model"], B=sp["B"], seeds=seeds, rng_key=sp["key"],
                         **prm))
        host.append((ptr, src))
    log(f"[batch] c3 full: {len(jobs)} jobs, {sum(h[1].size for h in host)} arcs")
    batch = fsg.Batch(jobs)
    infos, total_ms = batch.run()
    log(f"[batch] c3 full: {total_ms:.1f} ms device, tail-mode steps "
        f"{sum(int(x.tail_steps) for x in infos)} of {sum(int(x.steps_run) for x in infos)}")
    assert sum(int(x.tail_steps) for x in infos) > 0
    for i, (j, (ptr, src)) in enumerate(zip(jobs, host)):
        prm = {k: j[k] for k in ("p", "ic_prob", "beta", "gamma", "max_steps") if k in j}
        st, cnt, steps, absorbed = fsg.simulate(j["graph"], j["model"], j["seeds"], j["B"],
                                                j["rng_key"], **prm)
        assert torch.equal(batch.states[i], st), f"job {i} states differ from its solo run"
        assert torch.equal(batch.counts[i], cnt), f"job {i} counts differ from its solo run"
        assert (int(infos[i].steps_run), int(infos[i].absorbed)) == (steps, absorbed), i
        del st, cnt
        r0 = j["B"] // 3
        rs, _, _, _ = oracle_run((ptr, src), j["model"], j["seeds"], 2, j["rng_key"],
                                 replicate_offset=r0, **prm)
        got = batch.states[i][:, r0:r0 + 2].cpu().numpy()
        assert (got == rs).all(), f"job {i} ({j['model']}) sampled replicates differ from the oracle"
    log(f"[batch] c3 full: all {len(jobs)} jobs match their solo runs and the oracle samples")
    batch.close()
    for j in jobs:
        j["graph"].close()
