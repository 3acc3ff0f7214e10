"""Pins of the oracle's ablation freezing rules (Section 4.3, Table 3:
"+mingrad" freezes the lowest 25% gradients, "+random" a random 25%) and of
its Philox4x64-10 generator.  All CPU."""
import math

import numpy as np
import pytest

import oracle as O


def _numpy_philox_block(key, counter):
    """The first 4 outputs of numpy's Philox4x64-10 bit generator started
    at `counter` (numpy advances the counter by one before its first block)."""
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(counter, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("key,counter", [
    ((0, 0), (0, 0, 0, 0)),
    ((0x123456789ABCDEF, 0xFEDCBA9876543210), (5, 7, 0, 0)),
    ((42, 0), (2 ** 64 - 1, 3, 0, 0)),          # the increment carries into word 1
    ((2 ** 64 - 1, 2 ** 64 - 1), (11, 2 ** 64 - 1, 9, 8)),
])
def test_philox_matches_numpy_bit_generator(key, counter):
    c = list(counter)
    c[0] = (c[0] + 1) % 2 ** 64
    if c[0] == 0:
        c[1] = (c[1] + 1) % 2 ** 64
    assert O.philox4x64_10(c, key) == _numpy_philox_block(key, counter)


def test_random_rule_extremes_rate_and_fresh_draws():
    assert O.random_threshold(0.25) == 1 << 30 and O.random_threshold(1.0) == 1 << 32
    assert O.random_threshold(0.0) == 0
    n = 20000
    assert O.freeze_random(50, 0.0, 5, 1).sum() == 0
    assert O.freeze_random(50, 1.0, 5, 1).sum() == 50
    a = O.freeze_random(n, 0.25, 5, 100)
    b = O.freeze_random(n, 0.25, 5, 150)
    sd = math.sqrt(n * 0.25 * 0.75)
    assert abs(int(a.sum()) - n / 4) < 5 * sd and abs(int(b.sum()) - n / 4) < 5 * sd
    both = int((a & b).sum())                    # independent draws: overlap ~ n / 16
    assert abs(both - n / 16) < 5 * math.sqrt(n / 16)
    assert np.array_equal(a, O.freeze_random(n, 0.25, 5, 100))
    assert not np.array_equal(a, O.freeze_random(n, 0.25, 6, 100))


def test_mingrad_hand_cases():
    F = O.FLT_MAX
    s = [0.3, 0.1, F, 0.1, 0.2, 0.5, 0.1]          # 6 candidates (index 2 never seen)
    assert list(np.flatnonzero(O.freeze_mingrad(s, 0.5))) == [1, 3, 6]       # m = 3, ties by index
    assert list(np.flatnonzero(O.freeze_mingrad(s, 0.34))) == [1, 3]         # m = floor(2.04) = 2
    assert list(np.flatnonzero(O.freeze_mingrad(s, 0.25))) == [1]            # m = 1
    assert list(np.flatnonzero(O.freeze_mingrad(s, 0.7))) == [1, 3, 4, 6]   # m = 4
    assert list(np.flatnonzero(O.freeze_mingrad(s, 1.0))) == [0, 1, 3, 4, 5, 6]
    assert O.freeze_mingrad(s, 0.0).sum() == 0
    assert O.freeze_mingrad([F, F], 0.5).sum() == 0
    assert O.freeze_mingrad([], 0.5).size == 0


def test_mingrad_equals_stable_argsort_with_ties():
    rng = np.random.default_rng(9)
    for n in (1, 7, 257, 3001):
        s = (np.round(rng.random(n) * 20) / 20).astype(np.float32)     # many equal values
        s[rng.random(n) < 0.1] = np.float32(O.FLT_MAX)
        cand = np.flatnonzero(s < np.float32(O.FLT_MAX))
        for f in (0.25, 0.5, 0.9):
            m = int(math.floor(f * float(cand.size)))
            ref = np.zeros(n, np.uint8)
            ref[cand[np.argsort(s[cand], kind="stable")[:m]]] = 1
            got = O.freeze_mingrad(s, f)
            assert np.array_equal(got, ref)
            assert int(got.sum()) == m
            if 0 < m < cand.size:
                assert s[got == 1].max() <= s[cand][got[cand] == 0].min()


def test_apply_freeze_modes():
    old = np.array([1, 0, 1, 0], np.uint8)
    cond = np.array([0, 0, 1, 1], np.uint8)
    assert list(O.apply_freeze(old, cond, 0)) == [1, 0, 1, 1]
    assert list(O.apply_freeze(old, cond, 1)) == [0, 0, 0, 0]
    assert list(O.apply_freeze(old, cond, 2)) == [0, 0, 1, 1]


def test_densify_noise_box_muller_hand_values_and_moments():
    """The split children's normals (Section 4.1 densification with the 3DGS
    split rule): the Box-Muller transform of Philox words, checked by hand
    for one column and by its moments over many."""
    w = O.philox4x64_10((3, 7, 1, 0), (11, 1))
    u = [((x >> 11) + 0.5) / 2.0 ** 53 for x in w]
    nz = O.densify_noise(4, 11, 7)[3:6, 3]
    r = math.sqrt(-2 * math.log(u[0]))
    assert nz[0] == pytest.approx(r * math.cos(2 * math.pi * u[1]), rel=1e-15)
    assert nz[1] == pytest.approx(r * math.sin(2 * math.pi * u[1]), rel=1e-15)
    assert nz[2] == pytest.approx(math.sqrt(-2 * math.log(u[2])) * math.cos(2 * math.pi * u[3]), rel=1e-15)
    z = O.densify_noise(4000, 5, 100)
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)
    assert abs(np.corrcoef(z[0], z[1])[0, 1]) < 5 / math.sqrt(4000)
    assert not np.array_equal(z, O.densify_noise(4000, 5, 101))
