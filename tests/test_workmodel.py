"""The paper's near-field work model (Sec. 3.2.3), by brute-force counting.

A cube split into k pieces per axis has corner, edge, face and interior
pieces with 7, 11, 17 and 26 neighbours; with B particles per piece the
direct work per piece is W_c = B(B-1)/2 + N_B B^2 ~ (N_B + 1/2) B^2, and the
paper prints the work ratios R(4/2) = 968/60 and R(16/8) = 95288/10392.
These counts also fix the near-field pair count the GPU plan reports
((3k - 2)^3 ordered leaf pairs on a full level) and the M2L pair count
((6k - 8)^3 - (3k - 2)^3), checked on the device in test_gpu_plan.py.
"""
import itertools

import numpy as np


def _neighbour_counts(k):
    idx = np.arange(k)
    X, Y, Z = np.meshgrid(idx, idx, idx, indexing="ij")
    cnt = np.zeros((k, k, k), dtype=int)
    for d in itertools.product((-1, 0, 1), repeat=3):
        if d == (0, 0, 0):
            continue
        ok = ((X + d[0] >= 0) & (X + d[0] < k) & (Y + d[1] >= 0) & (Y + d[1] < k)
              & (Z + d[2] >= 0) & (Z + d[2] < k))
        cnt += ok
    return cnt


def _work(k):
    return float((_neighbour_counts(k) + 0.5).sum())


def test_neighbour_classes():
    c = _neighbour_counts(5)
    vals, counts = np.unique(c, return_counts=True)
    assert dict(zip(vals.tolist(), counts.tolist())) == {7: 8, 11: 12 * 3, 17: 6 * 9, 26: 27}


def test_work_ratios_match_printed_values():
    assert _work(2) == 60.0 and _work(4) == 968.0
    assert _work(8) == 10392.0 and _work(16) == 95288.0
    assert round(_work(4) / _work(2), 2) == 16.13
    assert round(_work(16) / _work(8), 2) == 9.17


def test_pair_count_closed_forms():
    for k in (2, 4, 8, 16):
        near = (_neighbour_counts(k) + 1).sum()  # ordered pairs, self included
        assert near == (3 * k - 2) ** 3
        # children of the parent's neighbours, per axis
        t = np.arange(k)
        per_axis = sum(int(((np.arange(k) // 2 >= tt // 2 - 1) & (np.arange(k) // 2 <= tt // 2 + 1)).sum())
                       for tt in t)
        assert per_axis == 6 * k - 8
