"""Web-scale independent cascade at full size: R-MAT scale 26 (2^26 nodes,
2^30 arcs, duplicates and self-loops kept), weighted cascade, 50 seeds,
B = 64, run to absorption in the launch configuration the benchmark times
(the frontier-driven run on a workspace an earlier run left clear).
Every final state, every count, the step count and absorption are compared
with the live-edge BFS oracle (pinned to the plain synchronous loop nest on
smaller graphs), which computes the same result work-efficiently."""
import time

import numpy as np
import pytest

import oracle
from paper_2603_14895_amd import workloads as W
from tests.gpu_util import NTHREADS, log

pytestmark = pytest.mark.gpu


def test_c4_full_size_bit_exact():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_14895_amd import fsg
    t0 = time.time()
    c = W.config_c4(device="cuda")
    gr = c["graph"]
    ptr, src = gr.numpy()
    del gr
    c["graph"] = None
    torch.cuda.empty_cache()
    log(f"[webscale] graph n={ptr.size - 1} nnz={src.size} in {time.time() - t0:.1f}s")
    g = fsg.DeviceGraph(ptr, src, out=True)
    runs = {}
    for var in (3, 2):  # frontier-driven (the default here), then the streaming step
        sim = fsg.Simulation(g, "ic", c["B"], ic_prob="weighted_cascade", max_steps=-1,
                             schedule=dict(kernel_variant=var))
        if var == 3:
            # a run with another key first: the compared run then reuses the
            # workspace that run left clear
            sim.run(c["seeds"], c["rng_key"] ^ 0x5A5A)
        info = sim.run(c["seeds"], c["rng_key"])
        runs[var] = (sim.states.cpu().numpy(), sim.counts.cpu().numpy().astype(np.uint32),
                     int(info.steps_run), int(info.absorbed))
        del sim
        log(f"[webscale] gpu variant {var}: steps={runs[var][2]} absorbed={runs[var][3]} "
            f"spread={runs[var][1].sum() / c['B']:.1f} at {time.time() - t0:.1f}s")
    del g
    torch.cuda.empty_cache()
    assert (runs[3][0] == runs[2][0]).all() and (runs[3][1] == runs[2][1]).all()
    assert runs[3][2:] == runs[2][2:]
    gst, gcnt, steps, absorbed = runs[3]
    del runs
    rs, rc, _, rsteps, rabs = oracle.ic_live_edge(ptr, src, c["seeds"], c["B"], c["rng_key"],
                                                 ic_prob=oracle.IC_WEIGHTED_CASCADE,
                                                 nthreads=NTHREADS, verbose=True)
    log(f"[webscale] oracle done at {time.time() - t0:.1f}s")
    assert steps == rsteps and absorbed == rabs
    assert (gcnt == rc).all()
    n = ptr.size - 1
    chunk = 1 << 22
    for v0 in range(0, n, chunk):
        assert (gst[v0:v0 + chunk] == rs[v0:v0 + chunk]).all(), v0
