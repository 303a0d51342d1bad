"""The workloads some GPU parity tests rely on are where those tests say:
checked on the CPU, so that a change to the input generator cannot move a
test off the case it is meant to cover without failing here."""
import math

import numpy as np
import pytest

from tests._helpers import sft_block_workloads, slice_edge_workload


@pytest.mark.parametrize("side", ["in", "out"])
@pytest.mark.parametrize("coef", ["f32", "f16"])
def test_slice_edge_workloads_sit_at_the_capacity(coef, side):
    """The bound on D-hat-phi's spread across a 256-frequency x 8-spindown
    tile (from max |tau| and max Tdot T over sky points and SFT midpoints)
    lies 5 bins inside the slice capacity, or half a bin beyond it."""
    w = slice_edge_workload(coef, side)
    assert w.n_fd == 12 and w.n_f > 256 and w.dfdot > 0
    tau = (w.t_start + 0.5 * w.t_sft - w.t_ref)[None, :] + w.sky @ w.pos.T
    p = (1.0 + w.sky @ w.vel.T) * w.t_sft
    spread = (255 * w.df + w.dfdot * 7 * np.abs(tau).max()) * p.max()
    cap = 384 if coef == "f16" else 296
    width = 262 + math.ceil(spread - 255)
    if side == "in":
        assert width == cap - 1 and (width & ~3) - spread > 4.9
    else:
        assert width == cap + 1


def test_sft_block_workloads_span_three_blocks():
    ws = sft_block_workloads()
    assert [(w.n_sft + 511) // 512 for w in ws] == [3, 2, 1]
    assert all(w.n_fd % 8 == 1 for w in ws)          # a 4-spindown remainder table as well
