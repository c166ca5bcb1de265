"""Web-scale independent cascade at full size: R-MAT scale 26 (2^26 nodes,
2^30 arcs, duplicates and self-loops kept), weighted cascade, 50 seeds,
B = 64, run to absorption in the launch configuration the benchmark times.
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
    g = fsg.DeviceGraph(ptr, src)
    sim = fsg.Simulation(g, "ic", c["B"], ic_prob="weighted_cascade", max_steps=-1)
    info = sim.run(c["seeds"], c["rng_key"])
    gst = sim.states.cpu().numpy()
    gcnt = sim.counts.cpu().numpy().astype(np.uint32)
    steps, absorbed = int(info.steps_run), int(info.absorbed)
    del sim, g
    torch.cuda.empty_cache()
    log(f"[webscale] gpu steps={steps} absorbed={absorbed} spread={gcnt.sum() / c['B']:.1f} "
        f"at {time.time() - t0:.1f}s")
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
