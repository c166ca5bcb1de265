"""Hegselmann-Krause on the GPU against the oracle: final opinions bit for
bit, steps, convergence and per-replicate counts, over both lane layouts
(B % 4 == 0 and not), hub rows on either side of the 256-arc cut, the
degenerate cases, and one step at full size on sampled rows."""
import numpy as np
import pytest

import oracle
from paper_2603_14895_amd import workloads as W
from tests.gpu_util import NTHREADS, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(ptr, src, h0, eps, K, act=0.5, schedule=None):
    from paper_2603_14895_amd import fsg
    g = fsg.DeviceGraph(ptr, src)
    h, cnt, info = fsg.hk(g, h0, eps, K, act=act, schedule=schedule)
    got = (h.cpu().numpy(), cnt.cpu().numpy(), int(info.steps_run), int(info.absorbed))
    g.close()
    rh, rsteps, rconv = oracle.hk(ptr, src, h0, eps, K, nthreads=NTHREADS)
    want = (rh, (rh > np.float32(act)).sum(axis=0).astype(np.int32), rsteps, rconv)
    return got, want


def _same(got, want, what):
    gh, gc, gs, ga = got
    rh, rc, rs, ra = want
    assert gh.shape == rh.shape, what
    if not np.array_equal(gh.view(np.uint32), rh.view(np.uint32)):
        bad = np.argwhere(gh.view(np.uint32) != rh.view(np.uint32))
        v, r = bad[0]
        raise AssertionError(f"{what}: {len(bad)} opinions differ, first node {v} replicate {r}: "
                             f"gpu {gh[v, r]!r} oracle {rh[v, r]!r}")
    assert (gs, ga) == (rs, ra), (what, gs, ga, rs, ra)
    assert (gc == rc).all(), what


CASES = [
    # n, mean degree, B, eps, max steps
    (3000, 12.0, 1, 0.32, 40),
    (3000, 12.0, 3, 0.32, 40),
    (3000, 12.0, 64, 0.32, 40),
    (2500, 16.0, 100, 0.2, 30),
    (2000, 10.0, 260, 0.45, 30),
    (1500, 24.0, 256, 0.8, 25),
    (4000, 8.0, 8, 0.05, 50),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_hk_matches_oracle(case):
    n, deg, B, eps, K = CASES[case]
    gr = W.chung_lu(n, deg, 2.5, 1200 + case)
    ptr, src = gr.numpy()
    h0 = W.uniform_opinions(n, B, 1300 + case)
    got, want = _both(ptr, src, h0, eps, K)
    log(f"[hk] n={n} B={B} eps={eps}: max indeg {np.diff(ptr).max()}, steps {got[2]}, "
        f"converged {got[3]}")
    _same(got, want, f"case {case}")


def _hub_graph(seed):
    """Random sparse arcs plus rows of 256 (light), 257, 320 and 5000 in-arcs
    (hubs of 5, 5 and 79 tiles), with repeated arcs and a self-loop."""
    rng = np.random.default_rng(seed)
    n = 6000
    # random arcs into rows 20.. only, so rows 10..13 get exactly d in-arcs
    edges = [(int(u), int(v)) for u, v in
             zip(rng.integers(0, n, size=20000), rng.integers(20, n, size=20000))]
    for hub, d in ((10, 256), (11, 257), (12, 320), (13, 5000)):
        edges += [(int(u), hub) for u in rng.integers(0, n, size=d - 2)]
        edges += [(hub, hub), (int(edges[-1][0]), hub)]
    return W.from_edges(n, edges).numpy()


@pytest.mark.parametrize("B", [1, 5, 64, 65, 130])
def test_hk_hub_rows(B):
    ptr, src = _hub_graph(77)
    d = np.diff(ptr)
    assert d[10] == 256 and d[11] == 257 and d[12] == 320 and d[13] == 5000
    for eps in (0.25, 1.5):
        h0 = W.uniform_opinions(ptr.size - 1, B, 78 + B)
        got, want = _both(ptr, src, h0, eps, 12)
        _same(got, want, f"hub graph B={B} eps={eps}")


def test_hk_degenerate_cases():
    from paper_2603_14895_amd import fsg
    ptr, src = W.chung_lu(500, 6.0, 2.5, 9).numpy()
    h0 = W.uniform_opinions(500, 12, 10)
    # eps = 0: the first step changes nothing
    got, want = _both(ptr, src, h0, 0.0, 9)
    _same(got, want, "eps 0")
    assert got[2] == 1 and got[3] == 1 and np.array_equal(got[0], h0)
    # no steps
    got, want = _both(ptr, src, h0, 0.3, 0)
    _same(got, want, "max_steps 0")
    assert got[2] == 0 and got[3] == 0
    # no arcs; one node
    got, want = _both(np.zeros(4, np.int64), np.zeros(0, np.int32), h0[:3], 0.5, 5)
    _same(got, want, "no arcs")
    got, want = _both(np.array([0, 1], np.int64), np.array([0], np.int32), h0[:1, :7], 0.5, 5)
    _same(got, want, "one node with a self-loop")
    # the same bits whatever the host poll interval; a run that reaches an
    # exact fixed point stops there (with a self-loop on every node, eps 0.5
    # does so after 177 steps; without, averages can swing by an ulp forever)
    loops = W.from_edges(500, [(int(src[k]), v) for v in range(500) for k in range(ptr[v], ptr[v + 1])]
                         + [(v, v) for v in range(500)]).numpy()
    a, _ = _both(*loops, h0, 0.5, 400, schedule=dict(steps_per_sync=1))
    b, want = _both(*loops, h0, 0.5, 400, schedule=dict(steps_per_sync=7, time_kernels=1))
    _same(a, want, "sync 1")
    _same(b, want, "sync 7")
    assert want[3] == 1 and want[2] < 400
    # two clusters at distance > eps never meet (counts over act = 0)
    far = np.where(h0 > 0, F(0.9), F(-0.9)).astype(np.float32) + h0 * F(0.01)
    got, want = _both(ptr, src, far, 0.5, 30, act=0.0)
    _same(got, want, "two clusters")
    assert (got[1] == (h0 > 0).sum(axis=0)).all()
    g = fsg.DeviceGraph(ptr, src)
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(fsg.FsgError):
            fsg.hk(g, h0, bad, 3)
    g.close()


F = np.float32


def test_hk_full_size_first_step_sampled():
    """One step on a 1M-node Chung-Lu graph (mean degree 20) with B = 256 at
    the launch configuration the benchmark uses: sampled rows, the largest
    hubs included, against the oracle row by row; a 20-step run stays inside
    the initial opinion range and is reproduced bit for bit."""
    from paper_2603_14895_amd import fsg
    gr = W.chung_lu(1_000_000, 20.0, 2.5, 4242)
    ptr, src = gr.numpy()
    B = 256
    h0 = W.uniform_opinions(ptr.size - 1, B, 4243)
    g = fsg.DeviceGraph(ptr, src)
    h1, _, info = fsg.hk(g, h0, 0.32, 1, want_counts=False)
    d = np.diff(ptr)
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([np.argsort(d)[-24:], rng.integers(0, d.size, 600),
                                     np.nonzero((d == 256) | (d == 257))[0][:8]]))
    want = oracle.hk_rows(ptr, src, h0, 0.32, rows)
    got = h1[rows].cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    log(f"[hk] full size: {rows.size} sampled rows (max indeg {d.max()}) match the oracle")
    hA, _, ia = fsg.hk(g, h0, 0.32, 20, want_counts=False, schedule=dict(steps_per_sync=4))
    hB, _, ib = fsg.hk(g, h0, 0.32, 20, want_counts=False)
    assert int(ia.steps_run) == int(ib.steps_run)
    assert torch_equal(hA, hB)
    lo, hi = float(h0.min()), float(h0.max())
    assert float(hA.min()) >= lo and float(hA.max()) <= hi
    g.close()


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a.view(torch.int32), b.view(torch.int32)))


def _both_w(ptr, src, h0, eps, mu, K, act=0.5):
    from paper_2603_14895_amd import fsg
    g = fsg.DeviceGraph(ptr, src)
    h, cnt, info = fsg.hk(g, h0, eps, K, act=act, mu=mu)
    got = (h.cpu().numpy(), cnt.cpu().numpy(), int(info.steps_run), int(info.absorbed))
    g.close()
    rh, rsteps, rconv = oracle.whk(ptr, src, h0, eps, mu, K, nthreads=NTHREADS)
    want = (rh, (rh > np.float32(act)).sum(axis=0).astype(np.int32), rsteps, rconv)
    return got, want


@pytest.mark.parametrize("mu", [0.2, 0.65, 0.0, 1.0])
@pytest.mark.parametrize("B", [1, 64, 130])
def test_whk_matches_oracle(mu, B):
    """Weighted HK (each node moves the fraction mu towards its HK mean; the
    parameters (0.32, 0.2) the paper compares): opinions bit for bit on a
    graph with hub rows (block-per-row path) and ordinary rows, mu = 0 (no
    move) and mu = 1 (plain HK) included."""
    ptr, src = _hub_graph(91)
    h0 = W.uniform_opinions(ptr.size - 1, B, 92 + B)
    got, want = _both_w(ptr, src, h0, 0.32, mu, 15)
    _same(got, want, f"whk mu={mu} B={B}")
    if mu == 1.0:
        hk_got, _ = _both(ptr, src, h0, 0.32, 15)
        assert np.array_equal(hk_got[0].view(np.uint32), got[0].view(np.uint32))
