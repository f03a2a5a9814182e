"""GPU tests of the Monte Carlo detector simulator (Section 2.1 physics,
compared with the Markov model as in Section 3.5).

The simulator and the oracle's counter-based simulator take the same
sampling steps on the same Philox4x32-10 streams, so their histograms agree
count for count.  (Only a pulse time that lands within a few units in the
last place of a bin edge or of a rearm instant could be decided differently,
since the GPU's log and cos may round differently from the host's; at these
sizes that has a probability far below 1e-6.)"""
import numpy as np
import pytest
import torch

from oracle import dtm as odtm, mc_philox, montecarlo as omc
from synth import scenes as sc

from gpu_helpers import lib, split

pytestmark = pytest.mark.gpu


def _mc(scenes, runs, cycles, burn, seed, lanes=0, segments=1):
    d = lib()
    plan = d.Plan(scenes, "f64", d.opts(tol=1e-10))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    hist, over = plan.mc_histograms(runs, cycles, burn, seed, lanes, segments_per_run=segments)
    torch.cuda.synchronize()
    out = split(hist.cpu().numpy().view(np.uint32).astype(np.int64), plan.pi_offsets), over.cpu().numpy()
    plan.close()
    return out


def _edge_scenes():
    return np.concatenate([
        sc.scene(period=100.0, dead_time=75.0, center=30.0, sigma=2.0, signal=2.0, background=0.5, n_bins=32),
        sc.scene(dead_time=0.0, center=40.0, sigma=3.0, signal=1.5, background=1.0, n_bins=7),
        sc.scene(dead_time=250.0, center=60.0, sigma=1.0, signal=3.0, background=0.7, n_bins=64),
        sc.scene(dead_time=20.0, center=1.0, sigma=2.0, signal=2.5, background=0.3, n_bins=100),
        sc.scene(dead_time=95.0, center=30.0, sigma=0.5, signal=12.0, background=6.0, n_bins=16),
        sc.scene(dead_time=33.3, signal=0.0, background=3.0, n_bins=5),
        sc.scene(dead_time=75.0, center=30.0, sigma=0.5, signal=3.0, background=0.0, n_bins=2),
    ])


@pytest.mark.parametrize("runs,cycles,burn,seed,lanes,segments", [
    (3, 400, 40, 2024, 0, 1), (3, 400, 40, 2024, 1, 1), (3, 397, 40, 2024, 64, 1), (3, 401, 5, 2024, 8, 1),
    (70, 30, 0, (7 << 32) | 99, 1, 1), (70, 30, 0, (7 << 32) | 99, 2, 1), (70, 30, 29, (7 << 32) | 99, 16, 1),
    (3, 400, 40, 2024, 0, 7), (3, 400, 40, 2024, 8, 400), (3, 401, 5, 2024, 64, 13), (3, 397, 40, 2024, 16, 2),
    (70, 30, 0, (7 << 32) | 99, 1, 30), (70, 30, 29, (7 << 32) | 99, 2, 3), (3, 2000, 100, 5, 0, 0)])
def test_histograms_match_oracle_count_for_count(runs, cycles, burn, seed, lanes, segments):
    """Edge cases: no dead time, dead time over two periods, pulses cut at
    t = 0, many photons per period (sorting), no signal, no background, two
    bins, ragged bin counts, run blocks that are not full (70 runs), period
    counts that are not a multiple of the lanes per run, one counted period,
    and a key that uses both seed words; every lane grouping gives the same
    counts.  Cut runs (segments > 1, 0 = automatic) give them too: from
    one-period segments, where most segment starts must be repaired and many
    repairs never meet the speculative walk (dead time over two periods, 18
    photons a period), to a ragged last segment and the burn-in inside it."""
    scenes = _edge_scenes()
    got, over = _mc(scenes, runs, cycles, burn, seed, lanes, segments)
    ref = mc_philox.histograms(scenes, runs, cycles, burn, seed)
    assert not over.any()
    for p, (g, r) in enumerate(zip(got, ref)):
        assert g.sum() > 0, p
        np.testing.assert_array_equal(g, r, err_msg=f"pixel {p}")


def test_segmented_runs_give_the_sequential_counts():
    """The Section 3.5 grid (S, B in {0.1, 3, 6, 9}) at 2^10 bins, 100 runs of
    5000 periods: the counts do not depend on how the runs are cut."""
    scenes = sc.paper_grid(dead_time=75.0, n_bins=1024)
    ref, _ = _mc(scenes, 100, 5000, 50, 11, 0, 1)
    for segments in (0, 2, 50, 777, 5000):
        got, over = _mc(scenes, 100, 5000, 50, 11, 0, segments)
        assert not over.any()
        for p, (g, r) in enumerate(zip(got, ref)):
            np.testing.assert_array_equal(g, r, err_msg=f"segments {segments} pixel {p}")


def test_pixel_and_run_streams_are_distinct():
    s = sc.scene(dead_time=50.0, signal=2.0, background=1.0, n_bins=64)
    got, _ = _mc(np.concatenate([s, s]), 5, 200, 0, 1)
    assert not np.array_equal(got[0], got[1])
    one, _ = _mc(s, 1, 200, 0, 1)
    ref = mc_philox.histograms(s, 1, 200, 0, 1)[0]
    np.testing.assert_array_equal(one[0], ref)


def test_rejects_unsupported_arguments():
    d = lib()
    s = sc.scene(dead_time=50.0, signal=20.0, background=5.0, n_bins=64)
    plan = d.Plan(s, "f64", d.opts(tol=1e-10))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    with pytest.raises(d.DtmError):
        plan.mc_histograms(4, 100, 0, 1)  # S + B > 24
    plan.close()
    s = sc.scene(dead_time=50.0, signal=2.0, background=1.0, n_bins=64)
    plan = d.Plan(s, "f64", d.opts(tol=1e-10))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.bind(ws)
    for runs, cycles, burn, lanes, segs in ((0, 100, 0, 0, 0), (4, 100, 100, 0, 0), (4, 0, 0, 0, 0),
                                            (4, 100, -1, 0, 0), (65536, 10, 0, 0, 0), (4, 1 << 32, 0, 0, 0),
                                            (1024, 65537, 1, 0, 0), (4, 100, 0, 3, 0), (4, 100, 0, 128, 0),
                                            (4, 100, 0, -1, 0), (4, 100, 0, 0, 101), (4, 100, 0, 0, -1)):
        with pytest.raises(d.DtmError):
            plan.mc_histograms(runs, cycles, burn, 1, lanes, segments_per_run=segs)
    # a scratch buffer shorter than the segment states
    short = torch.empty(plan.mc_scratch_bytes(4, 100, 10) - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(d.DtmError) as e:
        plan.mc_histograms(4, 100, 0, 1, 0, segments_per_run=10, scratch=short)
    assert e.value.status == d.DTM_ENOSPACE
    plan.close()


def test_markov_model_approaches_monte_carlo_as_bins_grow():
    """Section 3.5: the model's PDF at N bins, against a fine Monte Carlo
    histogram (2^10 bins, many runs) summed down to N bins, gets closer as N
    grows, down to a floor of O(1/N) plus the Monte Carlo noise.  (The
    independent NumPy simulator of the oracle, at 2e6 periods, puts the
    discretisation error of this scene at 2.8/N for N = 32 and below 2/N
    from N = 64 on; the bar here is 4/N.)"""
    base = dict(period=100.0, dead_time=75.0, center=30.0, sigma=2.0, signal=2.0, background=0.5)
    got, _ = _mc(sc.scene(n_bins=1024, **base), 1024, 20000, 100, 77, 0, 0)
    h = got[0].astype(np.float64)
    m = h.sum()
    errs = {}
    for n in (32, 64, 128, 256, 512, 1024):
        hn = h.reshape(n, 1024 // n).sum(axis=1) / m
        pi = odtm.stationary_pdf(sc.scene(n_bins=n, **base))
        errs[n] = np.abs(pi - hn).sum()
        assert errs[n] < omc.noise_floor_l1(n, m) + 4.0 / n, (n, errs[n])
    assert errs[32] > errs[64] > errs[128]
