"""The library's multi-DM pipeline pieces (Sec. 5.7; host code, no GPU)
against the oracle: the same DM trials, clusters and harmonic flags, entry
for entry, on random inputs with ties and on the boundaries of every rule;
and their argument errors."""
import numpy as np
import pytest

import paper_2004_03701_amd as ffa
from oracle import pipeline as op


@pytest.mark.parametrize("seed", range(25))
def test_dm_trials_equal_the_oracle(seed):
    g = np.random.default_rng(seed)
    n = int(g.integers(0, 3000))
    dms = np.sort(np.round(g.uniform(0, 2000, n), int(g.integers(0, 3))))
    f_lo = float(g.uniform(100, 1500))
    f_hi = f_lo * float(g.uniform(1.05, 3.0))
    smear = float(10 ** g.uniform(-5, -2))
    got = ffa.ffa_select_dm_trials(dms, f_lo, f_hi, smear)
    assert list(got) == op.select_dm_trials(dms, f_lo, f_hi, smear)


def test_dm_trials_at_exact_half_steps():
    # trials at multiples of half a step: differences at or next to the
    # boundary of the cover, decided the same way on both sides
    half = 0.5 * op.dm_step(1200.0, 1500.0, 1e-4)
    dms = np.arange(12) * half
    got = ffa.ffa_select_dm_trials(dms, 1200.0, 1500.0, 1e-4)
    assert list(got) == op.select_dm_trials(dms, 1200.0, 1500.0, 1e-4)


@pytest.mark.parametrize("seed", range(25))
def test_clusters_equal_the_oracle(seed):
    g = np.random.default_rng(1000 + seed)
    n = int(g.integers(0, 400))
    f = np.round(g.uniform(0.1, 5.0, n), int(g.integers(2, 5)))
    s = np.round(g.uniform(5, 15, n), 1).astype(np.float32)
    tol = float(g.choice([0.0, 1e-3, 1e-2, 0.05]))
    cl, br, mb = ffa.ffa_cluster_frequencies(f, s, tol)
    rc, rb, rm = op.cluster_frequencies(f, s, tol)
    assert np.array_equal(cl, rc) and np.array_equal(br, rb) and np.array_equal(mb, rm)


@pytest.mark.parametrize("seed", range(25))
def test_harmonic_flags_equal_the_oracle(seed):
    g = np.random.default_rng(2000 + seed)
    n = int(g.integers(0, 120))
    base = g.uniform(0.2, 3.0, 4)
    f = np.array([base[g.integers(0, 4)] * g.integers(1, 9) / g.integers(1, 9)
                  + g.normal(0, 2e-4) for _ in range(n)])
    s = np.round(g.uniform(5, 20, n), 0).astype(np.float32)  # ties in S/N
    tol = float(g.choice([1e-4, 5e-4, 2e-3]))
    order = int(g.integers(1, 10))
    got = ffa.ffa_flag_harmonics(f, s, tol, order)
    ref = op.flag_harmonics(f, s, tol, order)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_harmonic_flags_on_exact_ratios():
    # exact rational frequencies on a grid: the tolerance boundary is met
    f = np.array([0.5, 1.0, 1.5, 0.25, 0.75, 2.0, 0.375], dtype=np.float64)
    s = np.array([9, 9, 8, 8, 7, 7, 6], dtype=np.float32)
    for tol in (0.0, 1e-9, 0.125):
        got = ffa.ffa_flag_harmonics(f, s, tol, 8)
        ref = op.flag_harmonics(f, s, tol, 8)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def test_argument_errors():
    with pytest.raises(ffa.FFAError):
        ffa.ffa_select_dm_trials([2.0, 1.0], 1200, 1500, 1e-4)  # not ascending
    with pytest.raises(ffa.FFAError):
        ffa.ffa_select_dm_trials([1.0, 2.0], 1500, 1200, 1e-4)  # band reversed
    with pytest.raises(ffa.FFAError):
        ffa.ffa_select_dm_trials([1.0, np.nan], 1200, 1500, 1e-4)
    with pytest.raises(ffa.FFAError):
        ffa.ffa_cluster_frequencies([1.0, 2.0], [1.0, 2.0], -1.0)
    with pytest.raises(ffa.FFAError):
        ffa.ffa_cluster_frequencies([1.0, np.inf], [1.0, 2.0], 0.1)
    with pytest.raises(ffa.FFAError):
        ffa.ffa_flag_harmonics([1.0, 0.0], [1.0, 2.0], 0.1, 4)  # frequency must be > 0
    with pytest.raises(ffa.FFAError):
        ffa.ffa_flag_harmonics([1.0, 2.0], [1.0, 2.0], 0.1, 0)
    # empty inputs are fine
    assert ffa.ffa_select_dm_trials([], 1200, 1500, 1e-4).size == 0
    cl, br, mb = ffa.ffa_cluster_frequencies([], [], 0.1)
    assert cl.size == br.size == mb.size == 0
