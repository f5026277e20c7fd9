"""Plain CPU reference of the multi-DM pipeline pieces around the search
(Sec. 5.7): the choice of the DM trials to search, the grouping of the peaks
of all DM trials into clusters in frequency, and the flagging of clusters that
are harmonics of others.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may use it. It shares no
code with the library.

The paper names these steps without their rules; the readings taken here (and
by the library) are:
  * DM step (the classical rule the paper points to: limit the smearing of a
    pulse dedispersed at a wrong DM): a DM error dDM delays the top of the band
    against the bottom by k_DM * dDM * (f_lo^-2 - f_hi^-2), k_DM = 4.148808e3
    s MHz^2 pc^-1 cm^3; the step is the dDM whose half gives the largest
    allowed smearing: step = 2 * max_smear / (k_DM * (f_lo^-2 - f_hi^-2)).
  * DM trials searched: the fewest of the given (ascending) trials such that
    every given trial lies within step / 2 of a searched one.
  * Clusters: peaks of all DM trials, ordered by frequency, belong to one
    cluster while consecutive ones are at most tol apart in frequency (single
    linkage in frequency; DM and width play no part). A cluster's parameters
    are those of its brightest member (the lowest index among equal S/N).
    Clusters are numbered in ascending frequency.
  * Harmonics: cluster j is flagged a harmonic of cluster i when i is brighter
    (higher S/N, or equal S/N and a lower index) and, for coprime n, m in
    [1, max_order] other than n = m = 1, |nu_j - (n / m) nu_i| <= tol (1 + n / m)
    (the frequency uncertainty tol of each, the fundamental's scaled by n / m).
    The parent is the brightest such i; its ratio the one of smallest n + m,
    then smallest n.
"""
from __future__ import annotations

from math import gcd
from typing import List, Tuple

import numpy as np

K_DM = 4.148808e3  # s MHz^2 pc^-1 cm^3


def dm_step(f_lo_mhz: float, f_hi_mhz: float, max_smear_s: float) -> float:
    """The DM step whose half smears a pulse by max_smear_s across the band."""
    if not (0 < f_lo_mhz < f_hi_mhz) or not max_smear_s > 0:
        raise ValueError("need 0 < f_lo < f_hi and max_smear > 0")
    return 2.0 * max_smear_s / (K_DM * (f_lo_mhz ** -2 - f_hi_mhz ** -2))


def select_dm_trials(dms, f_lo_mhz: float, f_hi_mhz: float, max_smear_s: float) -> List[int]:
    """Indices of the trials to search: the fewest that leave every given trial
    within half a step of a searched one. Greedy from the lowest DM: the first
    trial not yet covered is covered by the highest trial at most half a step
    above it, which then covers every trial up to half a step above itself
    (for points on a line this choice is optimal)."""
    d = [float(v) for v in dms]
    if any(b < a for a, b in zip(d, d[1:])):
        raise ValueError("DM trials must ascend")
    half = 0.5 * dm_step(f_lo_mhz, f_hi_mhz, max_smear_s)
    keep = []
    i = 0
    n = len(d)
    while i < n:
        j = i
        while j + 1 < n and d[j + 1] - d[i] <= half:
            j += 1
        keep.append(j)
        k = j
        while k < n and d[k] - d[j] <= half:
            k += 1
        i = k
    return keep


def cluster_frequencies(freq, snr, tol: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Single-linkage clusters of points on the frequency axis: union-find
    over every pair closer than tol, written out pairwise. Returns the cluster
    of each point (clusters numbered by their lowest frequency), the brightest
    member of each cluster and its member count."""
    f = [float(v) for v in freq]
    s = [float(v) for v in snr]
    n = len(f)
    parent = list(range(n))

    def root(a):
        while parent[a] != a:
            a = parent[a]
        return a

    for a in range(n):
        for b in range(a + 1, n):
            if abs(f[a] - f[b]) <= tol:
                ra, rb = root(a), root(b)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
    groups = {}
    for a in range(n):
        groups.setdefault(root(a), []).append(a)
    order = sorted(groups.values(), key=lambda g: min((f[a], a) for a in g))
    cluster_of = np.empty(n, dtype=np.int64)
    brightest = np.empty(len(order), dtype=np.int64)
    members = np.empty(len(order), dtype=np.int64)
    for c, g in enumerate(order):
        for a in g:
            cluster_of[a] = c
        brightest[c] = min(g, key=lambda a: (-s[a], a))
        members[c] = len(g)
    return cluster_of, brightest, members


def flag_harmonics(freq, snr, tol: float, max_order: int):
    """Parent (or -1) and ratio n / m of every cluster, by trying every pair of
    clusters and every ratio."""
    f = [float(v) for v in freq]
    s = [float(v) for v in snr]
    n = len(f)
    parent = np.full(n, -1, dtype=np.int64)
    num = np.zeros(n, dtype=np.int64)
    den = np.zeros(n, dtype=np.int64)
    ratios = [(a, b) for a in range(1, max_order + 1) for b in range(1, max_order + 1)
              if gcd(a, b) == 1 and (a, b) != (1, 1)]
    ratios.sort(key=lambda r: (r[0] + r[1], r[0]))

    def brighter(i, j):
        return s[i] > s[j] or (s[i] == s[j] and i < j)

    for j in range(n):
        best = None
        for i in range(n):
            if i == j or not brighter(i, j):
                continue
            for a, b in ratios:
                if abs(f[j] - a / b * f[i]) <= tol * (1.0 + a / b):
                    if best is None or brighter(i, best[0]):
                        best = (i, a, b)
                    break
        if best is not None:
            parent[j], num[j], den[j] = best
    return parent, num, den
