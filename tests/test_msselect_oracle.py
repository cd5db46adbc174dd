"""CPU pins of the oracle for selection over sorted sequences (Appendix A,
msSelect; §4.3, amsSelect).

  * ms_select equals brute-force rank counting on small inputs with ties;
  * the rates of Algorithm "approxMusel" maximise the success probability
    of the geometric estimator (checked by a grid search: the mathematics,
    not the printed formula, decides);
  * the proof's closed form of that probability equals its sum, and tends
    to 1/e - e^(-kmax/kmin) as the proof states;
  * the max-based rate is the min-based rate of the mirrored range;
  * ams_check accepts exactly the valid flexible-k results.
"""
import math

import numpy as np
import pytest

import oracle
import synth

M = oracle.msselect


def sorted_rows(lens, gen, largest=False):
    off = np.zeros(len(lens) + 1, np.uint64)
    off[1:] = np.cumsum(lens)
    keys = gen(int(off[-1]))
    for r in range(len(lens)):
        a, b = int(off[r]), int(off[r + 1])
        seg = np.sort(keys[a:b], kind="stable")
        keys[a:b] = seg[::-1] if largest else seg
    return keys, off


@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("gen", ["alpha3", "u32", "f32"])
def test_ms_select_equals_brute_force(gen, largest):
    g = {"alpha3": lambda n: synth.small_alphabet_u32(n, 3, 5),
         "u32": lambda n: synth.uniform_u32(n, 6),
         "f32": lambda n: synth.normal_f32(n, 7)}[gen]
    lens = [0, 5, 1, 17, 9, 0, 30, 2]
    keys, off = sorted_rows(lens, g, largest)
    assert M.rows_sorted(keys, off, largest)
    n = int(off[-1])
    for k in (1, 2, n // 2, n - 1, n):
        kth, split = M.ms_select(keys, off, k, largest)
        sel, bkth = oracle.select_brute(keys, k, largest)
        assert kth == bkth and int(split.sum()) == k
        # the selection is a prefix of every row
        want = np.zeros(len(lens), np.int64)
        for x in sel:
            want[np.searchsorted(off.astype(np.int64), int(x), side="right") - 1] += 1
        assert np.array_equal(split, want)
        for r in range(len(lens)):
            a = int(off[r])
            assert set(range(a, a + int(split[r]))) <= set(sel.tolist())


@pytest.mark.parametrize("kmin,kmax", [(10, 20), (100, 400), (2, 3), (1000, 1001), (50, 5000)])
def test_min_rate_maximises_success(kmin, kmax):
    rho = M.ams_rho_min(kmin, kmax)
    best = M.geometric_success(rho, kmin, kmax)
    for r in np.linspace(1e-6, 0.999, 20001):
        assert M.geometric_success(r, kmin, kmax) <= best + 1e-12
    assert 0 < rho < 1


def test_success_probability_forms():
    for kmin, kmax in ((10, 20), (64, 1024), (3, 7)):
        for rho in (0.01, 1.0 / kmin, 0.3):
            assert M.geometric_success(rho, kmin, kmax) == \
                pytest.approx(M.geometric_success_sum(rho, kmin, kmax), rel=1e-9)
        # the proof's closed form for x = kmin
        assert M.success_probe_kmin(kmin, kmax) == \
            pytest.approx(M.geometric_success(1.0 / kmin, kmin, kmax), rel=1e-9)
    # and its limit 1/e - e^(-kmax/kmin)
    for ratio in (1.5, 2, 4):
        kmin = 10**6
        assert M.success_probe_kmin(kmin, int(ratio * kmin)) == \
            pytest.approx(1 / math.e - math.exp(-ratio), abs=1e-5)


def test_max_rate_is_the_mirrored_min_rate():
    for n, kmin, kmax in ((1000, 900, 990), (10**6, 10**6 - 500, 10**6 - 10), (50, 10, 40)):
        assert M.ams_rho_max(n, kmin, kmax) == \
            pytest.approx(M.ams_rho_min(n - kmax + 1, n - kmin + 1), rel=1e-12)


def test_ams_check():
    keys, off = sorted_rows([10, 20, 5], lambda n: synth.normal_f32(n, 3))
    _, s7 = M.ms_select(keys, off, 7)
    assert M.ams_check(keys, off, 5, 9, s7) == 0
    assert M.ams_check(keys, off, 8, 9, s7) == 1
    bad = s7.astype(np.int64).copy()
    i = int(np.argmax(bad))
    j = (i + 1) % 3
    bad[i] -= 1
    bad[j] += 1
    assert M.ams_check(keys, off, 5, 9, bad) == 2
