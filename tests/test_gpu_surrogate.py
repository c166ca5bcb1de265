"""What the trained surrogate gains over the method without it, end to end
at reduced size.
- Labels come from the simulator.
- The ensemble is trained on the GPU.
- The spread calibration is fitted on the training queries.
- The acceptance gate is calibrated on one half of held-out queries, on a
  graph never trained on.
Then, on the other half: accepted estimates stay within 2% of a
4096-replicate Monte Carlo reference, rejected ones fall back to plain Monte
Carlo, and plain Monte Carlo reaching the surrogate's accuracy is slower."""
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

    n, gamma, K = 20000, 0.1, 200
    rng = np.random.default_rng(2026)
    data, tr_sets = [], []
    for gi in range(2):
        gr = W.chung_lu(n, 20.0, 2.5, 6100 + gi)
        g = fsg.DeviceGraph(*gr.numpy())
        rv = fsg.DeviceGraph(*W.reverse_graph(gr).numpy())
        sets = S.seed_sets(n, 300, rng, max_size=400)
        betas = rng.uniform(0.01, 0.05, size=len(sets))
        y, _, _ = S.mc_frequencies(g, sets, betas, gamma, K, 1024, 10_000 * (gi + 1))
        data.append((g, rv, S.masks_of(sets, n), list(betas), y))
        tr_sets.append(sets)
    ens = S.Ensemble(4, seed=9)
    ens.train(data, epochs=10, sets_per_step=8, lr=3e-3, progress_every=5)

    pr, lab, tb, tk = [], [], [], []
    for (g, _, masks, betas, y), sets in zip(data, tr_sets):
        pr.append(ens.predict_spreads(g, masks, np.array(betas)).mean(axis=0))
        lab.append(y.sum(dim=1).double().cpu().numpy())
        tb += list(betas)
        tk += [len(s) for s in sets]
    coef = S.fit_calibration(np.concatenate(pr), np.concatenate(lab), tb, tk)

    gt = fsg.DeviceGraph(*W.chung_lu(n, 20.0, 2.5, 6199).numpy())
    qs = S.seed_sets(n, 100, rng, max_size=400)
    qb = rng.uniform(0.01, 0.05, size=len(qs))
    qk = np.array([len(q) for q in qs])
    _, ref, _ = S.mc_frequencies(gt, qs, qb, gamma, K, 4096, 77_000)
    mean, unc = S.uncertainty(ens.predict_spreads(gt, S.masks_of(qs, n), qb))
    cal_sp = S.apply_calibration(mean, qb, qk, coef)
    raw = np.abs(mean - ref) / ref
    err = np.abs(cal_sp - ref) / ref
    cal, test = np.arange(0, 50), np.arange(50, 100)
    gate = S.calibrate_gate(cal_sp[cal], unc[cal], ref[cal], qk[cal], 0.02)
    gate["calib"] = list(coef)
    log(f"[surrogate] held-out rel err median raw {np.median(raw):.4f} calibrated "
        f"{np.median(err):.4f}; gate tau {gate['tau']:.4f} min_seeds {gate['min_seeds']}")

    est = fsg.SpreadEstimator(ens.members, gt, gamma=gamma, max_steps=K, B_fallback=1024,
                              gate=gate)
    acc_err, acc, n_fb, t_sur = [], [], 0, []
    for i in test:
        t0 = time.perf_counter()
        sp, u, fb = est.estimate(qs[i], qb[i], 5150 + int(i))
        dt = time.perf_counter() - t0
        if fb:
            n_fb += 1
        else:
            # the library applies the same calibration to the same ensemble mean
            assert abs(sp - cal_sp[i]) <= 1e-4 * cal_sp[i]
            acc_err.append(abs(sp - ref[i]) / ref[i])
            acc.append(int(i))
            log(f"[surrogate] accepted query {int(i)}: seeds {qk[i]}, beta {qb[i]:.4f}, "
                f"uncertainty {u:.4f}, error {acc_err[-1]:.4f}")
            t_sur.append(dt)
    log(f"[surrogate] accepted {len(acc_err)}/{len(test)}, fallback {n_fb}; "
        f"accepted err mean {np.mean(acc_err) if acc_err else -1:.4f} "
        f"max {np.max(acc_err) if acc_err else -1:.4f}")
    assert len(acc_err) >= 10
    assert np.max(acc_err) <= 0.02

    # plain Monte Carlo at increasing B on the accepted queries
    e_sur, ts = float(np.mean(acc_err)), float(np.median(t_sur))
    sim, speedup = {}, None
    for B in (16, 64, 256, 1024, 4096):
        errs, times = [], []
        for i in acc[:20]:
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
