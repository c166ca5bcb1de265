"""Shared helpers of the GPU tests: run the HIP path through the C-ABI binding
and the CPU oracle on the same seeded inputs."""
from __future__ import annotations

import os
import sys

import numpy as np

import oracle
from paper_2603_14895_amd import fsg

NTHREADS = int(os.environ.get("FSG_ORACLE_THREADS", "16"))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_run(graph_np, model, seeds, B, key, *, schedule=None, replicate_offset=0, out=False,
            **kw):
    ptr, src = graph_np
    g = fsg.DeviceGraph(ptr, src, out=out)
    st, cnt, steps, absorbed = fsg.simulate(g, model, seeds, B, key,
                                            replicate_offset=replicate_offset,
                                            schedule=schedule, **kw)
    out = (st.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32), steps, absorbed)
    g.close()
    return out


def oracle_run(graph_np, model, seeds, B, key, *, replicate_offset=0, **kw):
    ptr, src = graph_np
    okw = dict(kw)
    if "ic_prob" in okw and isinstance(okw["ic_prob"], str):
        okw["ic_prob"] = fsg.IC_PROBS[okw["ic_prob"]]
    return oracle.simulate(model, ptr, src, seeds, B, key, replicate_offset=replicate_offset,
                           nthreads=NTHREADS, **okw)


def assert_same(gpu, ref, what=""):
    gs, gc, gst, ga = gpu
    rs, rc, rst, ra = ref
    assert gs.shape == rs.shape, what
    if not (gs == rs).all():
        bad = np.argwhere(gs != rs)
        v, r = bad[0]
        raise AssertionError(f"{what}: {len(bad)} state mismatches, first at node {v} "
                             f"replicate {r}: gpu {gs[v, r]} oracle {rs[v, r]}")
    assert (gc == rc).all(), what
    assert gst == rst, (what, gst, rst)
    assert ga == ra, (what, ga, ra)
