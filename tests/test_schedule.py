"""The host schedule of Algorithm 1 (Section 3.2.1 eq. 5, Section 3.2.2 eq. 7,
Section 3.2.3, Section 4.1 "GSta Details"): the oracle's lifecycle pinned by
hand-written sequences taken from the text, then the trainer's schedule
(paper_2504_06716_amd.schedule) checked against the oracle for every
iteration.  All CPU."""
import random

import numpy as np
import pytest

import oracle as O
from paper_2504_06716_amd import schedule as Sch

U, R = O.ACT_UPDATE, O.ACT_RESET

# (warm-up, update period, reset period, wait, window end, total iterations, K_f)
PAPER = dict(warmup=3000, every=250, reset_every=2000, wait=500, window_end=10000)
C2 = dict(warmup=600, every=50, reset_every=400, wait=100, window_end=1800)


def _events(cfg, stop_iter=None, upto=None):
    upto = upto or cfg["window_end"] + 1
    out = {}
    for k in range(upto):
        a = O.freeze_action(k, cfg["warmup"], cfg["every"], cfg["reset_every"], cfg["wait"], cfg["window_end"],
                            stop_iter)
        if a != O.ACT_NONE:
            out[k] = a
    return out


def test_lifecycle_paper_scale_hand_sequence():
    # Section 4.1: updates every 250 from the 3K warm-up, reset every 2K with
    # 500 iterations of no re-freezing, window closing at 10K
    ev = _events(PAPER, upto=12000)
    expect = {3000: U, 3250: U, 3500: U, 3750: U,
              4000: R, 4500: U, 4750: U, 5000: U, 5250: U, 5500: U, 5750: U,
              6000: R, 6500: U, 6750: U, 7000: U, 7250: U, 7500: U, 7750: U,
              8000: R, 8500: U, 8750: U, 9000: U, 9250: U, 9500: U, 9750: U,
              10000: R}
    assert ev == expect


def test_lifecycle_c2_scale_hand_sequence():
    # the 2000-iteration reading: warm-up 600, update 50, reset 400 + wait 100, window end 1800
    ev = _events(C2, upto=2000)
    expect = {600: U, 650: U, 700: U, 750: U,
              800: R, 900: U, 950: U, 1000: U, 1050: U, 1100: U, 1150: U,
              1200: R, 1300: U, 1350: U, 1400: U, 1450: U, 1500: U, 1550: U,
              1600: R, 1700: U, 1750: U,
              1800: R}
    assert ev == expect


def test_lifecycle_early_stop_closes_window():
    # early stop after 5000 iterations: the map is reset before iteration 5000
    # and never updated again
    ev = _events(PAPER, stop_iter=5000, upto=12000)
    assert ev[5000] == R and max(ev) == 5000
    assert [k for k in ev if k > 4000] == [4500, 4750, 5000]
    # a stop before the warm-up: one reset, nothing else
    assert _events(PAPER, stop_iter=2000, upto=12000) == {2000: R}


def test_training_end_hand_values():
    # window closes (forced stop) at 10K of 30K: finetune K_f = 1K, then the end
    assert O.training_end(30000, 10000, None, 1000) == 11000
    assert O.training_end(30000, 10000, 7000, 1000) == 8000            # early stop at 7K
    assert O.training_end(30000, 10000, 12000, 1000) == 11000          # late stop: forced one first
    assert O.training_end(2000, 1800, None, 200) == 2000               # the c2 reading
    assert O.training_end(2000, 1800, 1000, 200) == 1200
    assert O.training_end(8000, 10000, None, 1000) == 8000             # window never closes
    assert O.training_end(2000, 1800, 1950, 200) == 2000               # forced stop at 1800 comes first
    assert O.training_end(2000, 2500, 1950, 200) == 2150              # finetune runs past K


def test_simulated_lifecycle_hand_case():
    # PSNR after k iterations: 20, 24, 24.1, 24.15 at evaluations every 100
    # iterations; eq. 7 holds after the 4th (gains 0.1 and 0.05 < 0.2)
    table = {100: 20.0, 200: 24.0, 300: 24.1, 400: 24.15, 500: 30.0}
    sim = O.simulate_lifecycle(2000, 150, 50, 10000, 0, 1800, 60, eval_every=100, psnr_at=table.__getitem__,
                               es_eps=0.2, plateau=O.PlateauLR(0.75, 1, 1.0))
    assert sim["stop_iter"] == 400
    assert sim["end"] == 460
    assert sim["psnrs"] == [20.0, 24.0, 24.1, 24.15]
    acts = {k: a for k, a in enumerate(sim["actions"]) if a != O.ACT_NONE}
    assert acts == {150: U, 200: U, 250: U, 300: U, 350: U, 400: R}
    # plateau: 24.1 and 24.15 do not beat the best (24) by more than 1 dB:
    # the second such evaluation scales the position LR by 0.75
    sc = sim["pos_scale"]
    assert sc[399] == 1.0 and sc[400] == 0.75 and sc[459] == 0.75


# ---------------------------------------------------------------------------
# The trainer's schedule against the oracle, every iteration
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cfg,K", [(PAPER, 30000), (C2, 2000),
                                   (dict(warmup=10, every=5, reset_every=30, wait=5, window_end=50), 60),
                                   (dict(warmup=7, every=3, reset_every=10, wait=4, window_end=41), 50)])
@pytest.mark.parametrize("stop", [None, "early", "late"])
def test_freeze_schedule_matches_oracle(cfg, K, stop):
    stop_iter = {None: None, "early": cfg["warmup"] + 3 * cfg["every"], "late": cfg["window_end"] + 7}[stop]
    fs = Sch.FreezeSchedule(total_iters=K, **cfg)
    for k in range(K + 1):
        a = fs.action(k, stop_iter)
        b = O.freeze_action(k, cfg["warmup"], cfg["every"], cfg["reset_every"], cfg["wait"], cfg["window_end"],
                            stop_iter)
        assert a == b, (k, a, b)
        for lin in (False, True):
            fs.linear = lin
            ks = fs.window_close(stop_iter)
            ex, er = fs.thresholds(k, ks)
            assert ex == pytest.approx(O.freeze_threshold(k, K, fs.eps_xyz0, ks, linear=lin), rel=1e-15)
            assert er == pytest.approx(O.freeze_threshold(k, K, fs.eps_rgb0, ks, linear=lin), rel=1e-15)
        fs.linear = False
    for f in (0, 100, 1000):
        assert Sch.training_end(K, cfg["window_end"], stop_iter, f) == O.training_end(K, cfg["window_end"],
                                                                                        stop_iter, f)


@pytest.mark.parametrize("stop_iter", [None, 900, 12000])
def test_densify_schedule_matches_oracle(stop_iter):
    ds = Sch.DensifySchedule(total_iters=30000, start=500, stop=15000, every=100, reset_every=3000)
    for k in range(0, 16000):
        d, r = O.densify_action(k, 500, 15000, 100, 3000, stop_iter)
        assert ds.densify_now(k, stop_iter) == d, k
        assert ds.reset_now(k, stop_iter) == r, k
        if k % 97 == 0:
            ks = ds.end(stop_iter)
            gx, gr = ds.thresholds(k, ks)
            assert gx == pytest.approx(O.freeze_threshold(k, 30000, 2e-4, ks), rel=1e-15)
            assert gr == pytest.approx(O.freeze_threshold(k, 30000, 1e-6, ks), rel=1e-15)


def test_early_stop_and_plateau_match_oracle_on_random_sequences():
    rnd = random.Random(7)
    for _ in range(200):
        n = rnd.randint(1, 12)
        seq = [20.0]
        for _ in range(n):
            seq.append(seq[-1] + rnd.choice([-0.3, 0.05, 0.15, 0.19, 0.21, 0.5, 1.2, 2.0]))
        for j in range(1, len(seq) + 1):
            assert Sch.early_stop(seq[:j], 0.2) == O.early_stop(seq[:j], 0.2)
        a, b = Sch.PlateauLR(0.75, 1, 1.0), O.PlateauLR(0.75, 1, 1.0)
        for x in seq:
            assert a.step(x) == b.step(x)


def test_trainer_bookkeeping_matches_simulated_lifecycle():
    """The Trainer's host logic (validation while the window is open, eq. 7,
    plateau scale, window close, finetune end) against the oracle's
    simulation, driven by a fixed PSNR table instead of renders."""
    from paper_2504_06716_amd.train import Trainer

    class Stub:
        """The host-side part of a Trainer: every method that decides the
        schedule is the Trainer's own; rendering, freezing and the device
        checks are replaced by records."""
        check_flags = lambda self, where: None
        _validate = Trainer._validate
        window_close = Trainer.window_close
        end_iter = Trainer.end_iter
        finished = Trainer.finished
        _after_step = Trainer._after_step

    table = {k: 20.0 + (0.9 if k < 400 else 0.1) * k / 100 for k in range(100, 2001, 100)}
    for es in (0.2, None):
        fs = Sch.FreezeSchedule(total_iters=2000, **C2)
        cfg = type("Cfg", (), dict(schedule=fs, iters=2000, finetune_iters=200, eval_every=100,
                                   early_stop_eps=es, plateau=Sch.PlateauLR(0.75, 1, 1.0)))()
        st = Stub()
        st.cfg, st.k, st.psnrs, st.stop_iter, st.pos_scale, st.scale_log = cfg, 0, [], None, 1.0, []
        st.use_sched = False
        st.val_views = [0]
        st.evaluate = lambda views, st=st: table[st.k]
        acts = []
        while not st.finished:
            acts.append(fs.action(st.k, st.stop_iter))      # what Trainer._freeze_step applies
            st.k += 1
            st._after_step()
        sim = O.simulate_lifecycle(2000, C2["warmup"], C2["every"], C2["reset_every"], C2["wait"],
                                   C2["window_end"], 200, eval_every=100, psnr_at=table.__getitem__,
                                   es_eps=es if es is not None else -1e9, plateau=O.PlateauLR(0.75, 1, 1.0))
        assert st.stop_iter == sim["stop_iter"]
        assert st.k == sim["end"]
        assert acts == sim["actions"]
        assert st.psnrs == sim["psnrs"]
        scale_at = np.ones(st.k)
        for k0, s in st.scale_log:
            scale_at[k0:] = s
        np.testing.assert_array_equal(scale_at, sim["pos_scale"])
    assert sim["stop_iter"] is None and sim["end"] == 2000
