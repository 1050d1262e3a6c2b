"""Hand-worked Algorithm 3 cases (Appendix E): one-column blocks along coordinate axes,
whose incremental estimates can be followed by hand. Shared by the oracle pins and the
GPU tests; the derivations are in the comments of each case."""
from __future__ import annotations

import math

import numpy as np


def axis(m, d, s):
    b = np.zeros((m, 1))
    b[d, 0] = s
    return b


def norm_order_case():
    # energies 100 (e1), 9 (e2), 4 (e3); r = 1, eps^2 = 0.09
    # increasing norm: block 2 first: D = 4,  E = 104, 4/104  = 0.038 <= 0.09, accepted;
    #                  block 1:       D = 13, E = 113, 13/113 = 0.115 >  0.09, rejected
    #                  (and again in the next pass): clusters [0, 2], [1]
    # decreasing norm: block 1 first: 9/109 = 0.083 accepted, then block 2: 13/113
    #                  rejected: clusters [0, 1], [2]
    m = 4
    return [axis(m, 0, 10.0), axis(m, 1, 3.0), axis(m, 2, 2.0)], 1, 0.3


def continue_case():
    # energies: 0: 100 (e1), 1: 36 (e2), 2: 40 (e1), 3: 45 (e3); r = 1, eps^2 = 0.25
    # pass 1 in increasing norm: 1 (36/136 = 0.265, rejected), 2 (along the kept axis:
    # D = 0, accepted, E = 140), then 3 against the new state (45/185 = 0.243, accepted);
    # pass 2: 1 gives D = 81, E = 221, 0.367, rejected: clusters [0, 2, 3], [1].
    # Restarting after the acceptance of 2 would take 1 first (36/176 = 0.205, accepted)
    # and then reject 3 (81/221): clusters [0, 2, 1], [3].
    m = 4
    return [axis(m, 0, 10.0), axis(m, 1, 6.0), axis(m, 0, math.sqrt(40.0)), axis(m, 2, math.sqrt(45.0))], 1, 0.5


def residual_case():
    # energies: 0: 100 (e1), 1: 9 (e2), 2: 12.25 (e3), 3: 16 (e2); r = 2, eps^2 = 0.1,
    # residual sort. Pass-start residuals against span{e1} are the norms: order 1, 2, 3.
    #   1: two axes kept, D = 0, accepted;
    #   2: energies {100, 9, 12.25}: e2 dropped, D = 9, E = 121.25, 0.074, accepted;
    #   3: e2 is no longer kept: {100, 12.25, 16}, e3 dropped, D = 21.25, E = 137.25,
    #      0.155, rejected (also in pass 2): clusters [0, 1, 2], [3].
    # Re-sorting the rest of the pass after the acceptance of 1 (residuals against
    # span{e1, e2}: block 3 -> 0, block 2 -> 12.25) would take 3 first (D = 0, accepted)
    # and then 2 (D = 12.25, E = 137.25, 0.089, accepted): one cluster [0, 1, 3, 2].
    m = 4
    return [axis(m, 0, 10.0), axis(m, 1, 3.0), axis(m, 2, 3.5), axis(m, 1, 4.0)], 2, math.sqrt(0.1)


def tie_case():
    # 4 e1 and 3 e2 with r = 1: D = 9, E = 25, so the relative error is 3/5 exactly
    # (every intermediate is an exact small integer); eps = 0.6 accepts at the tie
    m = 3
    return [axis(m, 0, 4.0), axis(m, 1, 3.0)], 1, 0.6
