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
    assert w.n_fd == (12 if coef == "f16" else 16) and w.n_f > 256 and w.dfdot > 0
    # the library runs blocks of 8 there (a 16-block's slice would be twice as wide)
    import paper_0904_1826_amd as P
    split = P.fstat_spindown_split(w.n_fd, coef16=coef == "f16", allow16=False)
    assert split.get(8, 0) >= 8, split
    tau = (w.t_start + 0.5 * w.t_sft - w.t_ref)[None, :] + w.sky @ w.pos.T
    p = (1.0 + w.sky @ w.vel.T) * w.t_sft
    spread = (255 * w.df + w.dfdot * 7 * np.abs(tau).max()) * p.max()
    cap = 384 if coef == "f16" else 296
    width = 262 + math.ceil(spread - 255)
    if side == "in":
        assert width == cap - 1 and (width & ~3) - spread > 4.9
    else:
        assert width == cap + 1


def test_sft_block_workloads_span_several_blocks():
    ws = sft_block_workloads()
    assert [(w.n_sft + 511) // 512 for w in ws] == [3, 2, 1]
    assert [(w.n_sft + 255) // 256 for w in ws] == [5, 3, 2]
    assert all(w.n_fd % 8 == 1 for w in ws)          # spindowns in blocks of two sizes as well


@pytest.mark.parametrize("edge,kappa", [("zero", 0.0), ("one", 1.0 - 2.0 ** -34)])
def test_kappa_edge_workloads_sit_on_the_edge(oracle_lib, edge, kappa):
    """Every (template, SFT) pair of the kappa-edge work units has exactly the
    stated offset (the oracle's canonical FP64 bin position), and the windows
    stay inside the band."""
    from tests._helpers import kappa_edge_workload
    w = kappa_edge_workload(edge)
    k, kap, _, dphi = oracle_lib.bins(w, oracle_lib.all_templates(w))
    assert np.all(kap == kappa), (kap.min(), kap.max())
    assert np.all(dphi - k == kappa)
    assert k.min() - w.dterms + 1 >= w.k_first and k.max() + w.dterms <= w.k_first + w.n_bins - 1
    oracle_lib.fstat(w, oracle_lib.all_templates(w, [0]))      # band check passes
