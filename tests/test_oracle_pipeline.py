"""Pins of the oracle's multi-DM pipeline pieces (Sec. 5.7).

The paper names the steps (a DM step from the classical smearing rule, peaks
of all DM trials grouped into clusters in frequency, harmonics flagged) but
gives no rule or worked example, so the pins are: the dispersion constant
recomputed from the physical constants; the DM-trial choice against an
exhaustive search for the fewest covering trials; the clusters against the
consecutive-gap characterisation of single linkage on a line; the harmonic
flags on hand-worked cases and against their defining condition.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import pipeline as op


def test_dispersion_constant_from_physical_constants():
    # t = e^2 / (8 pi^2 eps0 m_e c) * DM / f^2 (SI, DM as a column density);
    # 1 pc cm^-3 = 3.0857e22 m^-2 and f in MHz give s MHz^2 pc^-1 cm^3
    sc = pytest.importorskip("scipy.constants")
    k_si = sc.e ** 2 / (8 * math.pi ** 2 * sc.epsilon_0 * sc.m_e * sc.c)
    k = k_si * sc.parsec * 1e6 / 1e12
    assert abs(k / op.K_DM - 1) < 2e-6


def test_dm_step_inverts_the_smearing():
    f_lo, f_hi, smear = 1182.0, 1582.0, 64e-6
    step = op.dm_step(f_lo, f_hi, smear)
    # half a step of DM error smears by exactly the allowed amount
    assert math.isclose(op.K_DM * 0.5 * step * (f_lo ** -2 - f_hi ** -2), smear, rel_tol=1e-12)
    with pytest.raises(ValueError):
        op.dm_step(1500.0, 1200.0, smear)


def covers(dms, chosen, half):
    return all(any(abs(d - dms[c]) <= half for c in chosen) for d in dms)


@pytest.mark.parametrize("seed", range(40))
def test_dm_choice_is_a_smallest_cover(seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(1, 11))
    dms = np.sort(np.round(g.uniform(0, 20, n), 1))
    smear = float(g.uniform(2e-5, 4e-4))
    half = 0.5 * op.dm_step(1200.0, 1500.0, smear)
    keep = op.select_dm_trials(dms, 1200.0, 1500.0, smear)
    assert keep == sorted(set(keep))
    assert covers(dms, keep, half)
    best = next(r for r in range(1, n + 1)
                if any(covers(dms, c, half) for c in itertools.combinations(range(n), r)))
    assert len(keep) == best


def test_dm_choice_limits():
    dms = np.arange(0.0, 50.0, 1.0)
    assert op.select_dm_trials(dms, 1200.0, 1500.0, 1e-9) == list(range(50))  # tiny step: all
    assert len(op.select_dm_trials(dms, 1200.0, 1500.0, 10.0)) == 1              # huge step: one
    assert op.select_dm_trials([], 1200.0, 1500.0, 1e-4) == []
    with pytest.raises(ValueError):
        op.select_dm_trials([3.0, 1.0], 1200.0, 1500.0, 1e-4)


@pytest.mark.parametrize("seed", range(30))
def test_clusters_are_runs_of_small_gaps(seed):
    g = np.random.default_rng(100 + seed)
    n = int(g.integers(1, 60))
    f = np.round(g.uniform(1.0, 2.0, n), 3)  # rounding makes equal frequencies and exact gaps
    s = np.round(g.uniform(5, 10, n), 1).astype(np.float32)
    tol = float(g.choice([0.0, 0.004, 0.01, 0.05]))
    cl, br, mb = op.cluster_frequencies(f, s, tol)
    order = sorted(range(n), key=lambda a: (f[a], a))
    # consecutive peaks in frequency share a cluster exactly when their gap is <= tol
    for a, b in zip(order, order[1:]):
        assert (cl[a] == cl[b]) == (f[b] - f[a] <= tol)
    # clusters numbered in ascending frequency, counts and brightest members
    assert [cl[a] for a in order] == sorted(cl[a] for a in order)
    assert cl[order[0]] == 0 and mb.sum() == n
    for c in range(len(br)):
        idx = [a for a in range(n) if cl[a] == c]
        assert mb[c] == len(idx)
        top = max(s[a] for a in idx)
        assert br[c] == min(a for a in idx if s[a] == top)


def test_clusters_by_hand():
    f = [1.00, 1.03, 1.01, 2.0, 1.06, 5.0]
    s = [7.0, 9.0, 9.0, 8.0, 6.0, 7.5]
    cl, br, mb = op.cluster_frequencies(f, s, 0.025)
    # 1.00 - 1.01 - 1.03 chain (gaps 0.01, 0.02); 1.06 is 0.03 away
    assert list(cl) == [0, 0, 0, 2, 1, 3]
    assert list(br) == [1, 4, 3, 5]  # equal S/N 9: the lower index
    assert list(mb) == [3, 1, 1, 1]


def test_harmonics_by_hand():
    f = [1.0, 2.0005, 1.5, 1.0 / 3.0, 1.234, 0.5]
    s = [20.0, 10.0, 8.0, 5.0, 6.0, 30.0]
    par, num, den = op.flag_harmonics(f, s, 0.001, 8)
    # 0.5 Hz is the brightest: 1.0 is its second harmonic, 2.0005 its fourth
    # (within 0.001 * 5), 1.5 its third; 1/3 is 2/3 of it (n + m = 5) before
    # 1/3 of 1.0 (n + m = 4 but a fainter parent); 1.234 is nothing
    assert list(par) == [5, 5, 5, 5, -1, -1]
    assert list(zip(num, den)) == [(2, 1), (4, 1), (3, 1), (2, 3), (0, 0), (0, 0)]


def test_harmonic_ratio_preference_and_tolerance():
    f = [3.0, 2.0]
    s = [10.0, 5.0]
    par, num, den = op.flag_harmonics(f, s, 1e-9, 4)
    assert par[1] == 0 and (num[1], den[1]) == (2, 3)
    # out of tolerance: 2.0 + 3e-9 > 2 + 1e-9 * (1 + 2/3)
    par, _, _ = op.flag_harmonics([3.0, 2.0 + 3e-9], s, 1e-9, 4)
    assert par[1] == -1
    # max_order bounds the ratios: 7/1 is not tried at order 4
    par, _, _ = op.flag_harmonics([1.0, 7.0], [10.0, 5.0], 1e-6, 4)
    assert par[1] == -1


@pytest.mark.parametrize("seed", range(20))
def test_harmonic_flags_satisfy_their_definition(seed):
    g = np.random.default_rng(500 + seed)
    n = int(g.integers(2, 25))
    base = g.uniform(0.5, 2.0, 3)
    f = []
    for _ in range(n):
        b = base[g.integers(0, 3)]
        a, c = int(g.integers(1, 6)), int(g.integers(1, 6))
        f.append(b * a / c + g.normal(0, 1e-4))
    s = np.round(g.uniform(5, 20, n), 0)
    tol, order = 3e-4, 6
    par, num, den = op.flag_harmonics(f, s, tol, order)

    def brighter(i, j):
        return s[i] > s[j] or (s[i] == s[j] and i < j)

    for j in range(n):
        cands = [i for i in range(n) if i != j and brighter(i, j) and any(
            abs(f[j] - a / b * f[i]) <= tol * (1 + a / b)
            for a in range(1, order + 1) for b in range(1, order + 1)
            if math.gcd(a, b) == 1 and (a, b) != (1, 1))]
        if not cands:
            assert par[j] == -1
            continue
        top = cands[0]
        for i in cands[1:]:
            if brighter(i, top):
                top = i
        assert par[j] == top
        a, b = num[j], den[j]
        assert math.gcd(a, b) == 1 and 1 <= a <= order and 1 <= b <= order and (a, b) != (1, 1)
        assert abs(f[j] - a / b * f[top]) <= tol * (1 + a / b)
