"""What the trained surrogate gains over the method without it, end to end
at reduced size: labels from the simulator, ensemble training on the GPU,
uncertainty threshold calibrated on one half of held-out queries (on a graph
never trained on), then on the other half: accepted estimates stay within 2%
of a 4096-replicate Monte Carlo reference, rejected ones fall back to plain
Monte Carlo, and at the surrogate's accuracy plain Monte Carlo is slower."""
import time

import numpy as np
import pytest

from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def test_surrogate_gain_over_plain_mc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_14895_amd import fsg
    from paper_2603_14895_amd import surrogate as S
    from paper_2603_14895_amd import workloads as W

    n, gamma, K = 8000, 0.1, 200
    rng = np.random.default_rng(2026)
    data = []
    for gi in range(2):
        gr = W.chung_lu(n, 20.0, 2.5, 6100 + gi)
        g = fsg.DeviceGraph(*gr.numpy())
        rv = fsg.DeviceGraph(*W.reverse_graph(gr).numpy())
        sets = S.seed_sets(n, 160, rng, max_size=400)
        betas = rng.uniform(0.01, 0.05, size=len(sets))
        y, _, _ = S.mc_frequencies(g, sets, betas, gamma, K, 512, 10_000 * (gi + 1))
        data.append((g, rv, S.masks_of(sets, n), list(betas), y))
    ens = S.Ensemble(4, seed=9)
    ens.train(data, epochs=10, sets_per_step=8, lr=3e-3, progress_every=5)

    gt = fsg.DeviceGraph(*W.chung_lu(n, 20.0, 2.5, 6199).numpy())
    qs = S.seed_sets(n, 60, rng, max_size=400)
    qb = rng.uniform(0.01, 0.05, size=len(qs))
    _, ref, _ = S.mc_frequencies(gt, qs, qb, gamma, K, 4096, 77_000)
    mean, unc = S.uncertainty(ens.predict_spreads(gt, S.masks_of(qs, n), qb))
    err = np.abs(mean - ref) / ref
    cal, test = np.arange(0, 20), np.arange(20, 60)
    tau = S.calibrate_tau(mean[cal], unc[cal], ref[cal], 0.02)
    log(f"[surrogate] held-out rel err median {np.median(err):.4f}; tau {tau:.4f}")

    est = fsg.SpreadEstimator(ens.members, gt, gamma=gamma, max_steps=K, B_fallback=1024, tau=tau)
    acc_err, n_fb, t_sur = [], 0, []
    for i in test:
        t0 = time.perf_counter()
        sp, u, fb = est.estimate(qs[i], qb[i], 5150 + int(i))
        dt = time.perf_counter() - t0
        if fb:
            n_fb += 1
        else:
            acc_err.append(abs(sp - ref[i]) / ref[i])
            t_sur.append(dt)
    log(f"[surrogate] accepted {len(acc_err)}/{len(test)}, fallback {n_fb}; "
        f"accepted err mean {np.mean(acc_err) if acc_err else -1:.4f} "
        f"max {np.max(acc_err) if acc_err else -1:.4f}")
    assert len(acc_err) >= 4
    assert np.mean(acc_err) <= 0.02

    # plain Monte Carlo at increasing B: time and error on the same queries
    e_sur, ts = float(np.mean(acc_err)), float(np.median(t_sur))
    sim = {}
    speedup = None
    for B in (16, 32, 64, 128, 256, 512, 1024, 2048):
        errs, times = [], []
        for i in test:
            t0 = time.perf_counter()
            _, cnt, _, _ = fsg.simulate(gt, "sir", qs[i], B, 9100 + int(i), beta=qb[i], gamma=gamma,
                                        max_steps=K, want_states=False)
            s = float(cnt.sum().item()) / B
            times.append(time.perf_counter() - t0)
            errs.append(abs(s - ref[i]) / ref[i])
        sim[B] = (float(np.mean(errs)), float(np.median(times)))
        if sim[B][0] <= e_sur:
            speedup = sim[B][1] / ts
            break
    log(f"[surrogate] surrogate {ts * 1e3:.2f} ms/query at err {e_sur:.4f}; MC "
        + ", ".join(f"B={b}: err {e:.4f} {t * 1e3:.2f} ms" for b, (e, t) in sim.items()))
    if speedup is None:  # no B tried reached the surrogate's accuracy
        speedup = max(t for _, t in sim.values()) / ts
    log(f"[surrogate] speed-up over plain MC at matched accuracy: {speedup:.1f}x")
    assert speedup > 1.0
