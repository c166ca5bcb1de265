"""Parity of the HIP path with the CPU oracle, bit for bit: final states,
per-node counts, steps run and absorption, on the same seeded inputs.

Sizes are chosen so the oracle finishes in seconds while spanning many tiles,
heavy-row segments and ragged replicate tails; the full-size SIR workload is
checked on replicates the oracle computes one by one.
"""
import numpy as np
import pytest

import oracle
from paper_2603_14895_amd import workloads as W
from tests.gpu_util import assert_same, gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_14895_amd import fsg
    fsg.lib()


def _both(gnp, model, seeds, B, key, what, **kw):
    log(f"[parity] {what} model={model} B={B} kw={ {k: v for k, v in kw.items() if k != 'edge_p'} }")
    g = gpu_run(gnp, model, seeds, B, key, **kw)
    kw.pop("schedule", None)
    kw.pop("out", None)
    r = oracle_run(gnp, model, seeds, B, key, **kw)
    assert_same(g, r, what)
    return g


def test_device_philox_matches_kat_and_oracle():
    import torch
    from paper_2603_14895_amd import fsg
    kat = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2),
           ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0])]
    for ctr, key in kat:
        c = torch.tensor(np.array(ctr, dtype=np.uint32).view(np.int32), device="cuda")
        o = torch.empty(4, dtype=torch.int32, device="cuda")
        fsg.fsg_philox4x32_10(c.data_ptr(), key[0], key[1], o.data_ptr(), 1)
        torch.cuda.synchronize()
        assert list(o.cpu().numpy().view(np.uint32)) == oracle.philox4x32_10(ctr, key)
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    c = torch.tensor(ctr.view(np.int32).ravel(), device="cuda")
    o = torch.empty(4096 * 4, dtype=torch.int32, device="cuda")
    fsg.fsg_philox4x32_10(c.data_ptr(), 0x1234, 0xABCD, o.data_ptr(), 4096)
    torch.cuda.synchronize()
    got = o.cpu().numpy().view(np.uint32).reshape(-1, 4)
    for i in range(0, 4096, 97):
        assert list(got[i]) == oracle.philox4x32_10(list(ctr[i]), [0x1234, 0xABCD])


def test_c1_ic_erdos_renyi_full():
    c = W.config_c1()
    gnp = c["graph"].numpy()
    _both(gnp, "ic", c["seeds"], c["B"], c["rng_key"], "c1", p=c["p"], max_steps=-1)


@pytest.mark.parametrize("ic_prob", ["uniform", "weighted_cascade", "per_edge"])
@pytest.mark.parametrize("B,offset", [(64, 0), (130, 3), (1, 7), (1024, 0), (1500, 5)])
def test_ic_variants(ic_prob, B, offset):
    gr = W.chung_lu(6000, 8.0, 2.5, 31)
    gnp = gr.numpy()
    ep = np.random.default_rng(4).uniform(0.0, 0.4, size=gr.nnz) if ic_prob == "per_edge" else None
    seeds = W.uniform_seeds(gr.n, 20, 32)
    _both(gnp, "ic", seeds, B, 0x1CE0 + B, f"ic-{ic_prob}", p=0.12, ic_prob=ic_prob, edge_p=ep,
          replicate_offset=offset, max_steps=-1)


@pytest.mark.parametrize("model", ["sir", "sis", "si"])
@pytest.mark.parametrize("B", [1024, 100])
def test_epidemics(model, B):
    gr = W.chung_lu(3000, 20.0, 2.5, 41)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 30, 42)
    _both(gnp, model, seeds, B, 0x5125 + B, model, beta=0.02, gamma=0.1, max_steps=40,
          replicate_offset=2 if B == 100 else 0)


@pytest.mark.parametrize("model", ["seir", "seis"])
@pytest.mark.parametrize("B,offset", [(1024, 0), (100, 2), (300, 0)])
def test_latent_epidemics(model, B, offset):
    """SEIR / SEIS: the aligned decision path (offset 0) and the general one
    (offset 2), one word per row and sixteen."""
    gr = W.chung_lu(3000, 20.0, 2.5, 45)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 30, 46)
    _both(gnp, model, seeds, B, 0x5E1A + B, model, beta=0.03, alpha=0.25, gamma=0.1,
          max_steps=50, replicate_offset=offset)


@pytest.mark.parametrize("model", ["seir", "seis"])
def test_latent_always_and_never(model):
    """alpha = 1 (every latent node turns infectious next step, no draw) and
    alpha = 0 (latent forever), beta = 1."""
    gr = W.chung_lu(800, 8.0, 2.5, 47)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 4, 48)
    for alpha, beta in ((1.0, 0.2), (0.0, 1.0), (0.5, 1.0)):
        _both(gnp, model, seeds, 192, 0x5E1B, f"{model} alpha={alpha}", beta=beta,
              alpha=alpha, gamma=0.3, max_steps=20)


@pytest.mark.parametrize("B", [200, 64])
def test_lt(B):
    gr = W.chung_lu(5000, 10.0, 2.5, 51)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 50, 52)
    _both(gnp, "lt", seeds, B, 0x17 + B, "lt", max_steps=-1, replicate_offset=1)


@pytest.mark.parametrize("model", ["ic", "sir", "lt", "sis", "seir"])
@pytest.mark.parametrize("sched", [
    dict(row_lanes=1, block_threads=64, tile_edges=64, heavy_threshold=16),
    dict(row_lanes=4, block_threads=1024, tile_edges=100000, heavy_threshold=40),
    dict(row_lanes=64, block_threads=128, tile_edges=500, heavy_threshold=7, steps_per_sync=1),
    dict(row_lanes=16, block_threads=512, tile_edges=3000, heavy_threshold=65535, steps_per_sync=64),
])
def test_schedules_and_heavy_rows(model, sched):
    """Every schedule -- lanes per row, block size, tile size, heavy-row cut
    (forcing many segments), host sync cadence -- gives identical bits."""
    gr = W.chung_lu(2500, 15.0, 2.5, 61)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 10, 62)
    K = -1 if model in ("ic", "lt") else 25
    _both(gnp, model, seeds, 300, 0xAB, f"sched-{sched}", p=0.1, beta=0.05, gamma=0.2,
          alpha=0.3, max_steps=K, schedule=sched, replicate_offset=9)


@pytest.mark.parametrize("model", ["ic", "sir", "lt", "seir"])
@pytest.mark.parametrize("sched", [
    None,
    dict(row_lanes=16, heavy_threshold=20, steps_per_sync=1),
    dict(row_lanes=64, block_threads=128, tile_edges=700, heavy_threshold=9, steps_per_sync=2),
])
def test_word_absorption_skip(model, sched):
    """With more than 16 words per node, a word none of whose replicates can
    change any more is left out of later steps (fewer lanes per row, more
    rows per wave, more edge lanes per heavy segment): same bits as the
    oracle, with heavy-row segments and the shortest host sync cadences (a
    word-flag ring of three slots)."""
    gr = W.chung_lu(1500, 12.0, 2.5, 71)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 3, 72)
    K = -1 if model in ("ic", "lt") else 60
    prm = dict(p=0.1, beta=0.05, gamma=0.2, alpha=0.3, max_steps=K)
    B = 1100
    g = _both(gnp, model, seeds, B, 0x3D0 + len(model), f"word-skip-{sched}", schedule=sched,
              replicate_offset=4, **prm)
    # the case is not vacuous: words stop changing at different steps
    okw = {k: v for k, v in prm.items() if k != "max_steps"}
    steps = [oracle_run(gnp, model, seeds, 64, 0x3D0 + len(model), replicate_offset=4 + 64 * w,
                        max_steps=K, **okw)[2] for w in range(0, B // 64, 4)]
    if model in ("ic", "lt"):
        assert len(set(steps)) > 1 and min(steps) < g[2], steps


@pytest.mark.parametrize("model", ["lt", "sir", "ic"])
@pytest.mark.parametrize("B", [1025, 4096, 4097])
def test_word_absorption_limits(model, B):
    """Word flags start at 17 words per node (1025 replicates, a one-replicate
    last word), end at 64 (4096 replicates: every lane of the wave holds a
    word flag) and are off from 65: all three give the oracle's bits."""
    gr = W.chung_lu(900, 10.0, 2.5, 81)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 2, 82)
    K = -1 if model in ("ic", "lt") else 40
    _both(gnp, model, seeds, B, 0x5EED + B, f"word-limits-{B}", p=0.1, beta=0.05, gamma=0.2,
          max_steps=K, replicate_offset=1)


@pytest.mark.parametrize("model", ["ic", "sir", "lt", "seir", "sis"])
@pytest.mark.parametrize("sched,B", [
    (dict(options=1), 300),
    (dict(options=1, row_lanes=1, block_threads=64, tile_edges=64, heavy_threshold=16), 300),
    (dict(options=1, row_lanes=4, heavy_threshold=40, steps_per_sync=3), 64),
    (dict(options=1, heavy_threshold=20, steps_per_sync=2), 1100),
])
def test_wide_offsets_path(model, sched, B):
    """The 64-bit-offset branches of the row-group kernels (taken by
    themselves only on graphs with n + 1 >= 2^24, (n + 1) W >= 2^29 or
    nnz >= 2^30), forced on small graphs: every model, edge-split rows,
    heavy-row segments and word absorption give the oracle's bits."""
    gr = W.chung_lu(2500, 15.0, 2.5, 63)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 8, 64)
    K = -1 if model in ("ic", "lt") else 30
    _both(gnp, model, seeds, B, 0xA1DE + B, f"wide-{sched}", p=0.1, beta=0.05, gamma=0.2,
          alpha=0.3, max_steps=K, schedule=sched, replicate_offset=5)


def test_lt_row_test_on_long_tails():
    """LT rows skip their count once at most half of the words are left and
    none of their in-neighbours gained an activation at the step before.  A
    directed path with a few random extra arcs makes cascades run for very
    different lengths across replicates, so most words stop long before the
    last one and the skip runs for many steps: same bits as the oracle."""
    n = 700
    rng = np.random.default_rng(91)
    extra = rng.integers(0, n, size=(900, 2))
    edges = [(i, i + 1) for i in range(n - 1)] + [(int(u), int(v)) for u, v in extra if u != v]
    gnp = W.from_edges(n, edges).numpy()
    seeds = np.array([0], dtype=np.int32)
    B, key = 2600, 0x7A1
    g = _both(gnp, "lt", seeds, B, key, "lt-long-tails", max_steps=-1, replicate_offset=8)
    steps = [oracle_run(gnp, "lt", seeds, 64, key, replicate_offset=8 + 64 * w, max_steps=-1)[2]
             for w in range(B // 64)]
    assert sorted(steps)[len(steps) // 2] + 10 < g[2], (sorted(steps), g[2])


def test_edge_cases():
    # self-loops, repeated arcs, isolated nodes, an in-star hub
    edges = [(0, 1), (0, 1), (1, 1), (1, 2), (2, 3), (3, 1), (5, 5)] + [(i, 6) for i in range(7, 40)]
    gr = W.from_edges(45, edges)
    gnp = gr.numpy()
    for model in ["ic", "sir", "si", "sis", "lt", "seir", "seis"]:
        for seeds, K in [([0, 7, 8, 0], 12), ([], 12), ([0, 3], 0), ([44], 5)]:
            for B in (1, 63, 65, 128):
                kw = dict(p=0.5, beta=0.4, gamma=0.3, alpha=0.6, max_steps=K)
                if model in ("ic", "lt") and K == 12:
                    kw["max_steps"] = -1
                _both(gnp, model, np.array(seeds, dtype=np.int32), B, 99 + B, f"edge-{model}",
                      **kw)
    # single node, no arcs
    gnp = W.from_edges(1, []).numpy()
    for model in ["ic", "sir", "lt"]:
        _both(gnp, model, np.array([0], dtype=np.int32), 70, 5, "n1", p=1.0, beta=1.0,
              gamma=1.0, max_steps=3 if model == "sir" else -1)
    # p = 1 and beta = 1 (the "always" sentinel), gamma = 1
    gr = W.chung_lu(500, 6.0, 2.5, 71)
    gnp = gr.numpy()
    _both(gnp, "ic", np.array([3], dtype=np.int32), 77, 1, "p1", p=1.0, max_steps=-1)
    _both(gnp, "sir", np.array([3], dtype=np.int32), 77, 2, "beta1", beta=1.0, gamma=1.0,
          max_steps=20)
    _both(gnp, "seir", np.array([3], dtype=np.int32), 77, 3, "seir-all-1", beta=1.0, alpha=1.0,
          gamma=1.0, max_steps=20)


def test_si_family_draw_classes_and_saturated_thresholds():
    """Every draw class of the SI-family decision: 1 to 15 infected
    in-neighbours (read from the code table), 16 or more (exact count),
    recovery and latent draws, and infection thresholds that saturate to
    'always' for large counts (beta = 0.95: k >= 13 rounds 1 - (1-beta)^k to
    1 in FP64, so those replicates take no draw).  Dense graphs and 10%
    initial infected put many replicates in every class at the first steps."""
    assert 1.0 - (1.0 - 0.95) ** 13 == 1.0 and 1.0 - (1.0 - 0.95) ** 12 < 1.0
    assert 1.0 - (1.0 - 0.5) ** 53 < 1.0 and 1.0 - (1.0 - 0.5) ** 54 == 1.0
    for gi, (n, deg) in enumerate(((1500, 40.0), (400, 120.0))):
        gr = W.chung_lu(n, deg, 2.5, 300 + gi)
        gnp = gr.numpy()
        seeds = W.uniform_seeds(n, n // 10, 310 + gi)
        for beta in (0.95, 0.5, 0.05):
            for model in ("sir", "sis", "si", "seir", "seis"):
                for B in (128, 100):
                    _both(gnp, model, seeds, B, 320 + B, f"classes-{model}-b{beta}",
                          beta=beta, gamma=0.3, alpha=0.4, max_steps=6)
            # replicate offsets not a multiple of four take the general path
            for off in (0, 2, 64):
                _both(gnp, "sir", seeds, 70, 330, f"classes-off{off}", beta=beta, gamma=0.3,
                      max_steps=6, replicate_offset=off)


@pytest.mark.parametrize("model", ["sir", "ic"])
def test_tail_mode_wide_rows(model):
    """Rows of more than 64 words (B = 4200, 66 words) in the tail mode: the
    counts that switch the mode read such a row with a whole wave.  The mode
    forced on, and left to its switch, gives the oracle's bits."""
    from paper_2603_14895_amd import fsg
    gr = W.chung_lu(900, 8.0, 2.5, 2201)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 15, 2202)
    if model == "sir":
        kw = dict(beta=0.08, gamma=0.2, max_steps=40)
        pull = {}
    else:
        kw = dict(p=0.1, ic_prob="uniform", max_steps=-1)
        pull = dict(kernel_variant=1)
    for sched in (dict(options=fsg.OPT_TAIL_ALWAYS, steps_per_sync=2), dict(steps_per_sync=3)):
        _both(gnp, model, seeds, 4200, 0x7B01, f"tail-wide-{model}-{sched}",
              schedule=dict(sched, **pull), out=True, **kw)


@pytest.mark.parametrize("model", ["sir", "sis", "si", "lt", "ic"])
def test_tail_mode(model):
    """The tail mode (a row that is not a candidate -- it and its
    in-neighbours hold no infected replicate (SI family) or no new activation
    (IC, LT) after step t-1, found from the out-arcs of the nodes that do -- is
    left out of step t) gives the oracle's bits: forced from the second chunk
    on, through the epidemic's growth or the cascade's bulk, with chunks of 1
    and 3 steps, ragged and full words, word flags (17 to 64 words), edge-split
    rows and heavy-row segments, and left to the library's own switch; a
    session stepped piece by piece in the tail mode ends in the same state.
    IC takes the mode on the pull step only (with one word per node and the
    out-adjacency bound, its default is the frontier-driven step)."""
    from paper_2603_14895_amd import fsg
    gr = W.chung_lu(3000, 10.0, 2.5, 2101)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 40, 2102)
    kw = dict(beta=0.05, gamma=0.2, max_steps=70 if model == "sir" else 25)
    if model == "lt":
        kw = dict(max_steps=-1)
    if model == "ic":
        kw = dict(p=0.09, ic_prob="uniform", max_steps=-1)
    always = fsg.OPT_TAIL_ALWAYS
    pull = dict(kernel_variant=1) if model == "ic" else {}
    # 1100 and 3000 replicates keep word flags (17 to 64 words)
    for B in (64, 100, 1024, 1100, 3000):
        for sched in (dict(options=always, steps_per_sync=1), dict(options=always, steps_per_sync=3),
                      dict(options=always, steps_per_sync=2, row_lanes=4, heavy_threshold=20),
                      dict(steps_per_sync=4), dict(options=fsg.OPT_TAIL_OFF)):
            _both(gnp, model, seeds, B, 0x7A11 + B, f"tail-{model}-{sched}",
                  schedule=dict(sched, **pull), out=True, **kw)
    # without the out-adjacency the mode is never taken
    _both(gnp, model, seeds, 100, 0x7A12, f"tail-{model}-no-out", out=False,
          schedule=dict(options=always, steps_per_sync=1), **kw)
    sess = fsg.Session(fsg.DeviceGraph(*gnp, out=True), model, seeds, 100, 0x7A77,
                       schedule=dict(options=always, steps_per_sync=1, **pull), **kw)
    try:
        for n in (1, 2, 5, 30, 40):
            info, _ = sess.step(n)
        st, cnt, _ = sess.read(want_states=True)
        got = (st.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32), int(info.steps_run),
               int(info.absorbed))
    finally:
        sess.close()
    r = oracle_run(gnp, model, seeds, 100, 0x7A77, **kw)
    assert_same(got, r, f"tail-session-{model}")


def test_replicate_split_and_repeat_invariance():
    """Splitting a batch with replicate_offset and repeating a run change
    nothing (counter-based draws keyed by the global replicate index)."""
    gr = W.chung_lu(4000, 12.0, 2.5, 81)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 40, 82)
    kw = dict(beta=0.03, gamma=0.1, max_steps=50)
    full = gpu_run(gnp, "sir", seeds, 256, 0xFEED, **kw)
    a = gpu_run(gnp, "sir", seeds, 101, 0xFEED, **kw)
    b = gpu_run(gnp, "sir", seeds, 155, 0xFEED, replicate_offset=101, **kw)
    assert (np.concatenate([a[0], b[0]], axis=1) == full[0]).all()
    again = gpu_run(gnp, "sir", seeds, 256, 0xFEED, schedule=dict(row_lanes=8), **kw)
    assert (again[0] == full[0]).all() and (again[1] == full[1]).all()


def test_c2_full_size_sampled_replicates():
    """The SIR workload at full size (Chung-Lu n = 10^6, mean degree 20,
    B = 1024, 200 steps) in the default schedule, with the out-adjacency
    bound as the benchmark binds it (so the late steps take the tail mode):
    replicates the oracle computes one by one, including ones whose
    generator block straddles a word boundary, match bit for bit; counts
    equal the states' tallies."""
    c = W.config_c2()
    gr = c["graph"]
    gnp = gr.numpy()
    log(f"[parity] c2 full n={gr.n} nnz={gr.nnz}")
    st, cnt, steps, absorbed = gpu_run(gnp, "sir", c["seeds"], c["B"], c["rng_key"], out=True,
                                       beta=c["beta"], gamma=c["gamma"], max_steps=c["max_steps"])
    assert (((st == 1) | (st == 2)).sum(axis=1) == cnt).all()
    for r0 in (0, 61, 1021):
        rs, _, _, _ = oracle_run(gnp, "sir", c["seeds"], 3, c["rng_key"], replicate_offset=r0,
                                 beta=c["beta"], gamma=c["gamma"], max_steps=c["max_steps"],
                                 want_states=True)
        assert (st[:, r0:r0 + 3] == rs).all(), r0
    log(f"[parity] c2 steps={steps} absorbed={absorbed} attack={(cnt.sum() / (gr.n * c['B'])):.4f}")


def _million_arc_hub():
    """A hub with 10^6 in-arcs (and 2000 out-arcs) on a sparse Chung-Lu
    background of 1.1e6 nodes."""
    import torch
    n, hub = 1_100_000, 7
    rng = np.random.default_rng(1717)
    base = W.chung_lu(n, 4.0, 2.5, 1718)
    bp, bs = base.numpy()
    bdst = np.repeat(np.arange(n, dtype=np.int64), np.diff(bp))
    srcs = rng.choice(n - 1, size=1_000_000, replace=False)
    srcs = srcs + (srcs >= hub)  # every node but the hub
    outs = rng.choice(n, size=2000, replace=False)
    src = np.concatenate([bs.astype(np.int64), srcs, np.full(outs.size, hub)])
    dst = np.concatenate([bdst, np.full(srcs.size, hub), outs])
    gr = W.pull_csr(n, torch.from_numpy(src), torch.from_numpy(dst), "hub1e6")
    assert int(gr.indeg()[hub]) >= 1_000_000
    return gr, hub


@pytest.mark.parametrize("model", ["sir", "lt", "seir", "ic"])
def test_million_arc_hub_sampled_replicates(model):
    """A row of 10^6 in-arcs (about a thousand heavy-row segments merged by
    the combine kernel, counts far past the SIR table's saturation, LT
    thresholds wider than the stored planes): replicates the oracle computes
    one by one match bit for bit."""
    gr, hub = _million_arc_hub()
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 3000, 1719)
    B, key = 256, 0x4B1B
    K = -1 if model in ("ic", "lt") else 25
    kw = dict(p=0.05, beta=0.02, gamma=0.1, alpha=0.4, max_steps=K)
    log(f"[parity] hub1e6 {model} n={gr.n} nnz={gr.nnz}")
    st, cnt, steps, absorbed = gpu_run(gnp, model, seeds, B, key, **kw)
    for r0 in (0, 125, 253):
        rs, _, _, _ = oracle_run(gnp, model, seeds, 3, key, replicate_offset=r0, want_states=True,
                                 **kw)
        assert (st[:, r0:r0 + 3] == rs).all(), (model, r0)
    log(f"[parity] hub1e6 {model}: steps={steps}, hub counted in {cnt[hub]} of {B}")


@pytest.mark.parametrize("ic_prob", ["uniform", "weighted_cascade", "per_edge"])
@pytest.mark.parametrize("sched", [
    dict(kernel_variant=2),
    dict(kernel_variant=2, tile_edges=300, heavy_threshold=50),
    dict(kernel_variant=2, tile_edges=100000, heavy_threshold=3, steps_per_sync=1),
])
@pytest.mark.parametrize("B,offset,K", [(64, 0, -1), (37, 5, -1), (64, 2, 3)])
def test_ic_edge_parallel(ic_prob, sched, B, offset, K):
    """The edge-parallel IC kernel (one word per node, frontier bitmap) gives
    the oracle's bits, including a step cap that leaves a live frontier."""
    gr = W.chung_lu(7000, 9.0, 2.5, 91)
    gnp = gr.numpy()
    ep = np.random.default_rng(9).uniform(0.0, 0.5, size=gr.nnz) if ic_prob == "per_edge" else None
    seeds = W.uniform_seeds(gr.n, 25, 92)
    _both(gnp, "ic", seeds, B, 0xED6E + B, f"ic-edge-{ic_prob}", p=0.15, ic_prob=ic_prob,
          edge_p=ep, replicate_offset=offset, max_steps=K, schedule=sched)


def _out_hub_graph():
    """Chung-Lu background plus a node with 5000 out-arcs (ten work items of
    the frontier-driven step) and one with 600."""
    rng = np.random.default_rng(93)
    base = W.chung_lu(6000, 6.0, 2.5, 94)
    bp, bs = base.numpy()
    dst = np.repeat(np.arange(base.n), np.diff(bp))
    edges = list(zip(bs.tolist(), dst.tolist()))
    for hub, k in ((11, 5000), (4321, 600)):
        edges += [(hub, int(v)) for v in rng.choice(base.n, size=k, replace=False) if v != hub]
    return W.from_edges(base.n, edges, "outhub")


@pytest.mark.parametrize("graph", ["chunglu", "outhub", "dense"])
@pytest.mark.parametrize("ic_prob", ["uniform", "weighted_cascade", "per_edge"])
@pytest.mark.parametrize("B,offset,K", [(64, 0, -1), (37, 5, -1), (64, 2, 3), (1, 0, -1)])
def test_ic_frontier_driven(graph, ic_prob, B, offset, K):
    """The frontier-driven IC step (kernel variant 3: work queues, pushes
    over out-arcs while the frontier has few of them, streams every arc
    otherwise) gives the oracle's bits: small frontiers (pushed), a node
    whose out-arcs span many work items, frontiers large enough to switch a
    run to streaming and back, ragged replicate counts, a step cap."""
    if graph == "chunglu":
        gr, p = W.chung_lu(7000, 9.0, 2.5, 95), 0.15
    elif graph == "outhub":
        gr, p = _out_hub_graph(), 0.2
    else:
        gr, p = W.erdos_renyi_directed(2000, 40.0, 96), 0.3
    gnp = gr.numpy()
    ep = np.random.default_rng(97).uniform(0.0, 0.5, size=gr.nnz) if ic_prob == "per_edge" else None
    seeds = np.concatenate([W.uniform_seeds(gr.n, 12, 98), [11, 11]]).astype(np.int32)
    _both(gnp, "ic", seeds, B, 0xF207 + B, f"ic-front-{graph}-{ic_prob}", p=p, ic_prob=ic_prob,
          edge_p=ep, replicate_offset=offset, max_steps=K, out=True,
          schedule=dict(kernel_variant=3, steps_per_sync=2 if K < 0 else 16))


def test_ic_frontier_driven_launch_widths():
    """A chunk of frontier-driven IC steps that starts from a pushable
    frontier launches fewer blocks than one that starts by streaming; on a
    graph large enough for the two widths to differ (20,000 nodes), a
    cascade that streams at its peak and pushes before and after gives the
    oracle's bits whether the width is chosen every step, every 3 steps or
    once for the whole run."""
    gr = W.erdos_renyi_directed(20000, 30.0, 131)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 8, 132)
    for spsync in (1, 3, 32):
        _both(gnp, "ic", seeds, 64, 0x51DE, f"ic-front-widths-sync{spsync}", p=0.12,
              ic_prob="uniform", max_steps=-1, out=True,
              schedule=dict(kernel_variant=3, steps_per_sync=spsync))


@pytest.mark.parametrize("B", [64, 50])
def test_ic_frontier_driven_workspace_reuse(B):
    """Runs after the first on one Simulation pass FSG_OPT_REUSE_WORKSPACE:
    each frontier-driven run that wrote outputs leaves its planes, bitmaps
    and ever-active plane clear (the finalize clears the ever-active words it
    read, a last pass the two frontiers no step cleared), so the next run
    skips clearing them.  Every run of a sequence -- different seeds and
    keys, step caps that stop a run with live frontiers, an empty seed set,
    runs to absorption, a counts-only run on its own object -- equals the
    oracle's, whether the tag was there or not."""
    from paper_2603_14895_amd import fsg
    gr = W.chung_lu(6000, 9.0, 2.5, 1717)
    gnp = gr.numpy()
    g = fsg.DeviceGraph(*gnp, out=True)
    runs = [(W.uniform_seeds(gr.n, 10, 1), 11, -1), (W.uniform_seeds(gr.n, 40, 2), 12, 3),
            (np.array([], dtype=np.int32), 13, -1), (W.uniform_seeds(gr.n, 5, 3), 14, 2),
            (W.uniform_seeds(gr.n, 25, 4), 15, -1), (W.uniform_seeds(gr.n, 25, 4), 15, -1)]
    for want_states in (True, False):
        sims = {}
        for i, (seeds, key, K) in enumerate(runs):
            # one object per step cap (the cap is a parameter of the object)
            if K not in sims:
                sims[K] = fsg.Simulation(g, "ic", B, schedule=dict(kernel_variant=3),
                                         want_states=want_states, p=0.12, max_steps=K)
            sim = sims[K]
            info = sim.run(seeds, key)
            r = oracle_run(gnp, "ic", seeds, B, key, p=0.12, max_steps=K)
            cnt = sim.counts.cpu().numpy().astype(np.uint32)
            assert (cnt == r[1]).all(), (i, want_states)
            assert (int(info.steps_run), int(info.absorbed)) == (r[2], r[3]), i
            if want_states:
                assert (sim.states.cpu().numpy() == r[0]).all(), i


def test_ic_rmat_weighted_cascade_vs_live_edge_bfs():
    """R-MAT (scale 18, edge factor 16, duplicates and self-loops kept),
    weighted cascade, 50 seeds, B = 64: the GPU matches the live-edge BFS
    oracle bit for bit, for both kernel variants."""
    gr = W.rmat(18, 16, 0.57, 0.19, 0.19, 1234)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 50, 1235)
    key = 0xC4C4C4C4
    rs, rc, _, rsteps, rabs = oracle.ic_live_edge(gnp[0], gnp[1], seeds, 64, key,
                                                 ic_prob=oracle.IC_WEIGHTED_CASCADE, nthreads=16)
    for var in (3, 2, 1):
        g = gpu_run(gnp, "ic", seeds, 64, key, ic_prob="weighted_cascade",
                    schedule=dict(kernel_variant=var), out=var == 3)
        assert_same(g, (rs, rc, rsteps, rabs), f"rmat18-variant{var}")
    log(f"[parity] rmat18 steps={rsteps} spread={rc.sum() / 64:.1f}")


@pytest.mark.parametrize("B,sched,beta", [(256, None, 0.06),
                                          (1024, dict(row_lanes=4, heavy_threshold=30), 0.06),
                                          (256, None, 0.95),
                                          (256, dict(heavy_threshold=30), 0.95)])
def test_sir_generator_call_count(B, sched, beta):
    """The counting run (FSG_OPT_COUNT_DRAWS) reports as many Philox4x32-10
    calls as the decision rule needs: at step t, one call per node and block
    of four replicates (g >> 2) in which some replicate needs a draw -- a
    susceptible one with k >= 1 infected in-neighbours (unless k <= 15 and
    1 - (1-beta)^k rounds to "always", as it does for k >= 13 at beta =
    0.95), or an infected one (gamma strictly
    between 0 and 1) -- counted here from the oracle's states after each
    step t - 1.  The states of the counting run equal the oracle's too."""
    import scipy.sparse as sp
    from paper_2603_14895_amd import fsg
    gr = W.chung_lu(900, 12.0, 2.5, 1811)
    ptr, src = gr.numpy()
    n = gr.n
    seeds = W.uniform_seeds(n, 12, 1812)
    key, kw = 0xD8A7, dict(beta=beta, gamma=0.25, max_steps=14)
    opt = dict(sched or {}, options=fsg.OPT_COUNT_DRAWS, time_kernels=0)
    g = fsg.DeviceGraph(ptr, src)
    sim = fsg.Simulation(g, "sir", B, schedule=opt, **kw)
    info = sim.run(seeds, key)
    got = (sim.states.cpu().numpy(), sim.counts.cpu().numpy().astype(np.uint32),
           int(info.steps_run), int(info.absorbed))
    assert_same(got, oracle_run((ptr, src), "sir", seeds, B, key, **kw), "counting run")
    dst = np.repeat(np.arange(n), np.diff(ptr))
    A = sp.csr_matrix((np.ones(src.size, dtype=np.int64), (dst, src)), shape=(n, n))
    table = oracle.sir_table(kw["beta"], int(np.diff(ptr).max()) + 1)
    always = 0xFFFFFFFF
    trec = oracle.thr(kw["gamma"])
    want = 0
    for t in range(1, int(info.steps_run) + 1):
        prev, _, _, _ = oracle_run((ptr, src), "sir", seeds, B, key, beta=kw["beta"],
                                   gamma=kw["gamma"], max_steps=t - 1)
        k = A @ (prev == 1).astype(np.int64)
        tk = table[np.minimum(k, table.size - 1)]
        need_s = (prev == 0) & (k >= 1) & ~((k <= 15) & (tk == always))
        need_i = (prev == 1) & (trec not in (0, always))
        want += int((need_s | need_i).reshape(n, B // 4, 4).any(axis=2).sum())
    log(f"[parity] generator calls B={B} beta={beta}: gpu {int(info.philox_calls)}, rule {want}")
    assert int(info.philox_calls) == want


@pytest.mark.parametrize("B,offset,K", [(256, 0, -1), (100, 2, -1), (1100, 1, -1), (64, 0, 3)])
@pytest.mark.parametrize("sched", [None, dict(row_lanes=4, heavy_threshold=25, steps_per_sync=2)])
def test_swir(B, offset, K, sched):
    """SWIR (susceptible, weakened, infected, removed): every state, count
    and step count equal the oracle's, with word absorption (1100
    replicates), unaligned generator blocks (offsets 1, 2), edge-split rows,
    heavy-row segments and a step cap."""
    gr = W.chung_lu(3000, 12.0, 2.5, 1901)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 15, 1902)
    _both(gnp, "swir", seeds, B, 0x5A1E + B, f"swir-{sched}", beta=0.08, alpha=0.12, gamma=0.3,
          max_steps=K, replicate_offset=offset, schedule=sched)
