"""Stateful stepping (run_iteration / run_iterations): a run cut into
session steps gives the same bits as one fsg_simulate call, and the per-step
state tallies equal the oracle's states counted at every step."""
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


CASES = [
    # model, n, mean degree, B, replicate offset, params, schedule
    ("sir", 2500, 12.0, 1024, 0, dict(beta=0.04, gamma=0.1, max_steps=40), None),
    ("sis", 1500, 8.0, 130, 2, dict(beta=0.06, gamma=0.2, max_steps=30), None),
    ("ic", 3000, 10.0, 64, 0, dict(p=0.08, max_steps=-1), None),           # edge-parallel kernel
    ("ic", 2000, 8.0, 200, 5, dict(p=0.1, ic_prob="weighted_cascade", max_steps=-1), None),
    ("lt", 2000, 10.0, 300, 0, dict(max_steps=-1), None),
    ("sir", 1800, 15.0, 256, 0, dict(beta=0.05, gamma=0.2, max_steps=25),
     dict(heavy_threshold=20, row_lanes=4)),
    ("seir", 2000, 12.0, 512, 0, dict(beta=0.05, alpha=0.3, gamma=0.15, max_steps=40), None),
    # more than 16 words per node: word flags kept across calls (two-step ring margin)
    ("lt", 1500, 10.0, 1100, 0, dict(max_steps=-1), dict(steps_per_sync=2)),
    ("sir", 1200, 12.0, 1300, 3, dict(beta=0.05, gamma=0.2, max_steps=60),
     dict(steps_per_sync=1, heavy_threshold=20)),
    ("swir", 2000, 12.0, 700, 1, dict(beta=0.08, alpha=0.15, gamma=0.4, max_steps=-1), None),
]


def _pieces(total):
    return [1, 3, 5, 2, total]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_session_resume_is_exact(case):
    from paper_2603_14895_amd import fsg
    model, n, deg, B, off, prm, sched = CASES[case]
    gr = W.chung_lu(n, deg, 2.5, 910 + case)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(n, 7, 920 + case)
    key = 0x5E55_0000 + case
    whole = gpu_run(gnp, model, seeds, B, key, replicate_offset=off, schedule=sched, **prm)
    g = fsg.DeviceGraph(*gnp)
    ss = fsg.Session(g, model, seeds, B, key, replicate_offset=off, schedule=sched, **prm)
    done = 0
    for k in _pieces(10_000):
        info, _ = ss.step(k)
        assert info.steps_run >= done
        done = int(info.steps_run)
        if info.absorbed:
            break
    st, cnt, _ = ss.read()
    got = (st.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32), int(info.steps_run),
           int(info.absorbed))
    ss.close()
    log(f"[session] {model} B={B}: steps {got[2]} absorbed {got[3]}")
    assert_same(got, whole, f"case {case} stepped vs one call")
    if B > 1024:
        assert_same(got, oracle_run(gnp, model, seeds, B, key, replicate_offset=off, **prm),
                    f"case {case} stepped vs oracle")


@pytest.mark.parametrize("case", [0, 2, 4, 6])
def test_session_tallies_match_oracle(case):
    """Tally after each step == (#state-1, #state-2) of the oracle's states at
    that step (the oracle run with max_steps = t)."""
    from paper_2603_14895_amd import fsg
    model, n, deg, B, off, prm, sched = CASES[case]
    n = 400
    gr = W.chung_lu(n, deg, 2.5, 930 + case)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(n, 5, 940 + case)
    key = 0x7A11_0000 + case
    T = 12
    g = fsg.DeviceGraph(*gnp)
    p = dict(prm)
    p["max_steps"] = T if model not in ("lt", "ic") else -1
    ss = fsg.Session(g, model, seeds, B, key, replicate_offset=off, **p)
    _, _, t0 = ss.read(want_states=False)
    seed_state = 2 if model in ("seir", "seis") else 1  # step 0: the seeds, infectious
    want0 = [0, 0, 0]
    want0[seed_state - 1] = len(np.unique(seeds)) * B
    assert t0 == tuple(want0)
    info, tal = ss.step(T, tally=True)
    ss.close()
    for t in range(1, T + 1):
        q = dict(prm)
        q["max_steps"] = t
        rs, _, rsteps, _ = oracle_run(gnp, model, seeds, B, key, replicate_offset=off, **q)
        want = (int((rs == 1).sum()), int((rs == 2).sum()), int((rs == 3).sum()))
        assert tuple(int(x) for x in tal[t - 1]) == want, (t, tal[t - 1], want, rsteps)
    log(f"[session] {model}: tallies of {T} steps match the oracle "
        f"(steps run {int(info.steps_run)}, absorbed {int(info.absorbed)})")


@pytest.mark.parametrize("B,off", [(64, 0), (50, 3)])
def test_session_frontier_driven_ic(B, off):
    """Frontier-driven IC (work queues over three rotating frontier planes):
    a run cut into session pieces equals one call and the oracle, and the
    per-step tallies equal the oracle's states counted at every step."""
    from paper_2603_14895_amd import fsg
    gr = W.chung_lu(5000, 9.0, 2.5, 931)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 9, 932)
    key, prm = 0xF5E5, dict(p=0.12, max_steps=-1)
    sched = dict(kernel_variant=3, steps_per_sync=3)
    whole = gpu_run(gnp, "ic", seeds, B, key, replicate_offset=off, schedule=sched, out=True, **prm)
    assert_same(whole, oracle_run(gnp, "ic", seeds, B, key, replicate_offset=off, **prm), "whole")
    g = fsg.DeviceGraph(*gnp, out=True)
    ss = fsg.Session(g, "ic", seeds, B, key, replicate_offset=off, schedule=sched, **prm)
    tallies = []
    for k in _pieces(10_000):
        info, t = ss.step(k, tally=True)
        tallies += [tuple(int(x) for x in row) for row in t]
        if info.absorbed:
            break
    st, cnt, _ = ss.read()
    got = (st.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32), int(info.steps_run),
           int(info.absorbed))
    assert_same(got, whole, "frontier-driven session vs one call")
    for step in range(1, min(len(tallies), whole[2]) + 1, 3):
        rs, _, _, _ = oracle_run(gnp, "ic", seeds, B, key, replicate_offset=off, max_steps=step,
                                 p=prm["p"])
        want = tuple(int((rs == s).sum()) for s in (1, 2, 3))
        assert tallies[step - 1] == want, step
    ss.close()
    g.close()


def test_session_frontier_driven_ic_launch_widths():
    """A frontier-driven IC session on a graph large enough for pushing and
    streaming chunks to get different grids (20,000 nodes; the cascade
    streams at its peak): the grid choice carried from piece to piece gives
    the same bits as one call and the oracle."""
    from paper_2603_14895_amd import fsg
    gr = W.erdos_renyi_directed(20000, 30.0, 141)
    gnp = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 8, 142)
    key, prm = 0x51DF, dict(p=0.12, max_steps=-1)
    sched = dict(kernel_variant=3, steps_per_sync=2)
    whole = gpu_run(gnp, "ic", seeds, 64, key, schedule=sched, out=True, **prm)
    assert_same(whole, oracle_run(gnp, "ic", seeds, 64, key, **prm), "whole")
    g = fsg.DeviceGraph(*gnp, out=True)
    ss = fsg.Session(g, "ic", seeds, 64, key, schedule=sched, **prm)
    for k in (1, 1, 3, 2, 5, 100):
        info, _ = ss.step(k)
        if info.absorbed:
            break
    st, cnt, _ = ss.read()
    got = (st.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32), int(info.steps_run),
           int(info.absorbed))
    assert_same(got, whole, "frontier-driven session (launch widths) vs one call")
    ss.close()
    g.close()
