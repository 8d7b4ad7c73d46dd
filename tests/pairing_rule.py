"""The time-reversal pairing rule of the paired transition lists, written
out for the tests: the partner of k is -k-q on the grid (Monkhorst-Pack
index r maps to N-1-r under k -> -k); a transition (k, n, m) is kept when
the partner index of k is larger, or when k is its own partner and n < m."""
import numpy as np


def partner(kgrid, qj):
    N = np.asarray(kgrid)
    idx = np.array(np.unravel_index(np.arange(np.prod(N)), N)).T
    rt = np.mod(N - 1 - idx - np.asarray(qj), N)
    return (rt[:, 0] * N[1] + rt[:, 1]) * N[2] + rt[:, 2]


def keep(k, n, m, kt):
    k, n, m = np.asarray(k), np.asarray(n), np.asarray(m)
    return (kt[k] > k) | ((kt[k] == k) & (n < m))
