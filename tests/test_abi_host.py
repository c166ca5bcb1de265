"""Host-side tests of the C-ABI (no GPU needed): the library loads, exports
every symbol the header declares, validates its arguments before touching the
device, and its row-tile planner keeps the load-balance bound of the paper's
target-node partition (Sec. 3.2, Proposition "Load Balance Guarantee")."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2603_14895_amd import fsg
from paper_2603_14895_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsg.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fsg_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported():
    lib = fsg.lib()
    names = _declared()
    assert "fsg_simulate" in names and "fsg_graph_create" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps every declared call
    assert set(names) <= set(fsg.exported_names())
    want = int(re.search(r"#define FSG_ABI_VERSION (\d+)", open(HEADER).read()).group(1))
    assert fsg.fsg_abi_version() == want


def _graph(n=50, seed=1):
    gr = W.chung_lu(n, 4.0, 2.5, seed)
    return gr.numpy()


def test_graph_create_validation():
    ptr, src = _graph()
    n, nnz = ptr.size - 1, src.size
    h = fsg.fsg_graph_create(n, nnz, ptr.ctypes.data, src.ctypes.data)
    assert fsg.fsg_graph_stats(h)[:2] == (n, nnz)
    fsg.fsg_graph_destroy(h)
    bad_src = src.copy()
    bad_src[3] = n
    with pytest.raises(fsg.FsgError) as e:
        fsg.fsg_graph_create(n, nnz, ptr.ctypes.data, bad_src.ctypes.data)
    assert e.value.code == fsg.FSG_EINVAL and "out of range" in str(e.value)
    bad_ptr = ptr.copy()
    bad_ptr[5], bad_ptr[6] = bad_ptr[6], bad_ptr[5] - 1
    with pytest.raises(fsg.FsgError):
        fsg.fsg_graph_create(n, nnz, bad_ptr.ctypes.data, src.ctypes.data)
    with pytest.raises(fsg.FsgError) as e:
        fsg.fsg_graph_create(0, 0, ptr.ctypes.data, None)
    assert e.value.code == fsg.FSG_EINVAL
    with pytest.raises(fsg.FsgError) as e:
        fsg.fsg_graph_create(n, nnz + 1, ptr.ctypes.data, src.ctypes.data)
    assert e.value.code == fsg.FSG_EINVAL
    with pytest.raises(fsg.FsgError) as e:
        fsg.fsg_graph_create(n, 2**31, ptr.ctypes.data, src.ctypes.data)
    assert e.value.code == fsg.FSG_EUNSUPPORTED


def test_arc_count_cap_is_refused_before_reading_arrays():
    """nnz above 2^31 - 256 is refused up front (kernels keep arc indices in
    int32 and look up to 256 positions past one); the arrays are not read."""
    for nnz in (2**31 - 255, 2**31 - 1):
        ptr = np.array([0, nnz], dtype=np.int64)
        src = np.zeros(4, dtype=np.int32)
        with pytest.raises(fsg.FsgError) as e:
            fsg.fsg_graph_create(1, nnz, ptr.ctypes.data, src.ctypes.data)
        assert e.value.code == fsg.FSG_EUNSUPPORTED and "2^31 - 256" in str(e.value)


def test_schedule_options_validated():
    ptr, src = _graph()
    n, nnz = ptr.size - 1, src.size
    h = fsg.fsg_graph_create(n, nnz, ptr.ctypes.data, src.ctypes.data)
    try:
        prm, _ = fsg.make_params("sir", beta=0.1, gamma=0.1, max_steps=5)
        for opt in (fsg.OPT_WIDE_OFFSETS, fsg.OPT_COUNT_DRAWS, fsg.OPT_REUSE_WORKSPACE,
                    fsg.OPT_TAIL_OFF, fsg.OPT_TAIL_ALWAYS, 7, 15, 23):
            ok = fsg.make_schedule({"options": opt})
            assert fsg.fsg_sim_workspace_size(h, prm, 64, ok) > 0
        # unknown bits, and the two tail-mode options together
        for bad in (32, 24, 1 << 30):
            with pytest.raises(fsg.FsgError) as e:
                fsg.fsg_sim_workspace_size(h, prm, 64, fsg.make_schedule({"options": bad}))
            assert e.value.code == fsg.FSG_EINVAL
    finally:
        fsg.fsg_graph_destroy(h)


def test_params_validation_before_any_launch():
    ptr, src = _graph()
    n, nnz = ptr.size - 1, src.size
    h = fsg.fsg_graph_create(n, nnz, ptr.ctypes.data, src.ctypes.data)
    try:
        cases = [
            (dict(model="sir", beta=0.1, gamma=0.1, max_steps=-1), 10, fsg.FSG_EINVAL),
            (dict(model="sir", beta=float("nan"), gamma=0.1, max_steps=5), 10, fsg.FSG_EINVAL),
            (dict(model="sis", beta=0.1, gamma=1.5, max_steps=5), 10, fsg.FSG_EINVAL),
            (dict(model="ic", p=-0.1), 10, fsg.FSG_EINVAL),
            (dict(model="ic", p=0.1), 0, fsg.FSG_EINVAL),
            (dict(model="ic", ic_prob="per_edge"), 10, fsg.FSG_EINVAL),
        ]
        for kw, B, code in cases:
            prm, _ = fsg.make_params(**kw)
            with pytest.raises(fsg.FsgError) as e:
                fsg.fsg_sim_workspace_size(h, prm, B, None)
            assert e.value.code == code, kw
        prm, _ = fsg.make_params("ic", ic_prob="per_edge", edge_p=np.full(nnz, 2.0))
        with pytest.raises(fsg.FsgError):
            fsg.fsg_sim_workspace_size(h, prm, 10, None)
        # bad schedules
        prm, _ = fsg.make_params("ic", p=0.1)
        for sd in [dict(row_lanes=3), dict(block_threads=96), dict(heavy_threshold=70000),
                   dict(steps_per_sync=-2)]:
            with pytest.raises(fsg.FsgError):
                fsg.fsg_sim_workspace_size(h, prm, 10, fsg.make_schedule(sd))
        ws = fsg.fsg_sim_workspace_size(h, prm, 100, None)
        assert ws > 0 and ws % 256 == 0
        # an unbound graph, bad seeds and small workspaces are refused on the host
        seeds = np.array([1, 2], dtype=np.int32)
        with pytest.raises(fsg.FsgError) as e:
            fsg.fsg_simulate(h, prm, seeds.ctypes.data, 2, 100, 0, 1, None, None, 0, None, None)
        assert e.value.code == fsg.FSG_EINVAL and "bound" in str(e.value)
    finally:
        fsg.fsg_graph_destroy(h)


def test_word_flag_ring_in_workspace():
    """Jobs with 17 to 64 words per node carry a word-flag ring of
    steps_per_sync + 2 slots of W flags; the others carry none.  Only the two
    flag rings depend on steps_per_sync, so the workspace difference between
    two cadences is the ring growth alone."""
    ptr, src = _graph()
    n, nnz = ptr.size - 1, src.size
    h = fsg.fsg_graph_create(n, nnz, ptr.ctypes.data, src.ctypes.data)
    try:
        prm, _ = fsg.make_params("ic", p=0.1)

        def a256(x):
            return (x + 255) // 256 * 256

        for W in (1, 2, 16, 17, 40, 64, 65):
            B = 64 * W - (W > 1)  # a ragged last word
            ws = [fsg.fsg_sim_workspace_size(h, prm, B, fsg.make_schedule(dict(steps_per_sync=k)))
                  for k in (1, 9)]
            job_ring = a256(10 * 4) - a256(2 * 4)
            word_ring = a256(11 * W * 4) - a256(3 * W * 4) if 16 < W <= 64 else 0
            assert ws[1] - ws[0] == job_ring + word_ring, W
    finally:
        fsg.fsg_graph_destroy(h)


def test_hk_entry_points_refuse_unbound_graphs_on_the_host():
    ptr, src = _graph()
    n, nnz = ptr.size - 1, src.size
    h = fsg.fsg_graph_create(n, nnz, ptr.ctypes.data, src.ctypes.data)
    try:
        for call in (lambda: fsg.fsg_hk_workspace_size(h, 8, None),
                     lambda: fsg.fsg_hk(h, 0.3, 5, 8, None, None, None, 0, 0.5, None,
                                        stream=ctypes.c_void_p(0)),
                     lambda: fsg.fsg_hk_workspace_size(None, 8, None)):
            with pytest.raises(fsg.FsgError) as e:
                call()
            assert e.value.code == fsg.FSG_EINVAL and "bound" in str(e.value)
    finally:
        fsg.fsg_graph_destroy(h)


@pytest.mark.parametrize("heavy", [10**9, 40])
@pytest.mark.parametrize("parts", [1, 3, 17, 64, 500])
def test_row_tiles_load_balance_bound(heavy, parts):
    """Every part's load is within w_max of the ideal W/d, parts are
    contiguous, non-empty and cover all rows."""
    gr = W.chung_lu(3000, 12.0, 2.5, 5)
    ptr, _ = gr.numpy()
    row_cost = 4
    b = fsg.fsg_plan_row_tiles(ptr, heavy, row_cost, parts)
    d = np.diff(ptr)
    w = np.where(d > heavy, 0, d) + row_cost
    assert b[0] == 0 and b[-1] == gr.n and (np.diff(b) > 0).all()
    assert len(b) - 1 <= parts
    loads = np.array([w[b[i]:b[i + 1]].sum() for i in range(len(b) - 1)])
    total, wmax = w.sum(), w.max()
    if len(loads) == parts:
        assert (np.abs(loads - total / parts) < wmax).all()
    else:
        # parts that would be empty are dropped; each load still stays below
        # the ideal plus one row
        assert (loads < total / parts + wmax).all()
    assert loads.sum() == total


def test_batch_plan_validation():
    ptr, src = _graph()
    n, nnz = ptr.size - 1, src.size
    h = fsg.fsg_graph_create(n, nnz, ptr.ctypes.data, src.ctypes.data)
    try:
        arr = (fsg.fsg_job * 1)()
        prm, _ = fsg.make_params("ic", p=0.1)
        arr[0].g = h
        arr[0].prm = prm
        arr[0].B = 10
        with pytest.raises(fsg.FsgError) as e:
            fsg.fsg_batch_plan(arr, 1, 8)  # graph not bound
        assert e.value.code == fsg.FSG_EINVAL and "job 0" in str(e.value)
        with pytest.raises(fsg.FsgError):
            fsg.fsg_batch_plan(arr, 0, 8)
        with pytest.raises(fsg.FsgError):
            fsg.fsg_batch_plan(arr, 1, 0)
    finally:
        fsg.fsg_graph_destroy(h)


def _run_injected(spec, code):
    """Runs `code` in a fresh interpreter with FSG_FAULT_INJECT=spec (the
    library reads it once per process) and returns its stdout lines."""
    import subprocess
    import sys
    env = dict(os.environ, FSG_FAULT_INJECT=spec)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return r.stdout.split()


_PRELUDE = """
import numpy as np
from paper_2603_14895_amd import fsg
ptr = np.array([0, 1, 2, 4], dtype=np.int64)
src = np.array([1, 2, 0, 1], dtype=np.int32)
def create():
    try:
        return fsg.fsg_graph_create(3, 4, ptr.ctypes.data, src.ctypes.data), 0
    except fsg.FsgError as e:
        return None, e.code
"""


def test_fault_injection_host_allocation():
    """FSG_FAULT_INJECT=alloc:2: the second guarded host allocation fails
    with FSG_ENOMEM and a message; the calls before and after succeed."""
    out = _run_injected("alloc:2", _PRELUDE + """
g1, c1 = create()
g2, c2 = create()
msg = fsg.fsg_last_error()
g3, c3 = create()
print(c1, c2, c3, 'host' in msg and 'allocation' in msg)
""")
    assert out == ["0", str(fsg.FSG_ENOMEM), "0", "True"]


def test_fault_injection_device_call():
    """FSG_FAULT_INJECT=device:1: the first checked HIP call (the upload in
    fsg_graph_bind) reports FSG_EDEVICE without calling HIP, so the path runs
    on a host without a GPU; nothing is marked bound."""
    out = _run_injected("device:1", _PRELUDE + """
g, c = create()
try:
    fsg.fsg_graph_bind(g, 1 << 20, 1 << 20, None)
    code = 0
except fsg.FsgError as e:
    code = e.code
msg = fsg.fsg_last_error()
prm, _ = fsg.make_params('ic', p=0.1)
try:
    fsg.fsg_sim_workspace_size(g, prm, 64, None)
    sim = 0
except fsg.FsgError as e:
    sim = e.code
print(code, 'injected' in msg, sim)
""")
    assert out[:2] == [str(fsg.FSG_EDEVICE), "True"]
