"""The flop model's time-node bookkeeping against the oracle's coefficient
tables: the nodes whose time-derivative weight is exactly zero (the model
leaves their flux evaluations and weighted terms out, as the forward kernels
skip them) are those where the oracle's exact-rational table holds 0."""
import numpy as np
import pytest

import oracle
from paper_2007_01416_amd import flops as F


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_weighted_time_nodes_match_the_oracle_tables(p):
    gt = np.asarray(oracle.coeffs(p)["gt"])      # gt[k][ri], node r = ri - p + 1
    r0 = p - 1
    for k in range(1, 2 * p):
        nz, nzf = F.time_nodes(p, k)
        assert nz == int(np.count_nonzero(gt[k]))
        assert nzf == nz - int(gt[k][r0] != 0)


def test_zero_weights_are_the_even_orders_at_the_last_node():
    # on the nodes -q+1..q the even-order weights of r = q vanish (one node fewer per even level)
    for q in range(2, 5):
        for k in range(1, 2 * q):
            nz, _ = F.time_nodes(q, k)
            assert nz == 2 * q - (1 if k % 2 == 0 else 0)


def test_counts_drop_exactly_the_skipped_terms():
    # q33: 2 of the 25 predicted-state flux evaluations per node are skipped (levels 3 and 5),
    # each a 2D Euler f, g pair (16 flops) and its 2 x 4 weighted fused multiply-adds (16 flops)
    full = 36 * 2 * (F.C_FG_EULER2D + 2 * 2 * 4)
    assert F.corner_flops_2d(3, 3) == 50838 - full
