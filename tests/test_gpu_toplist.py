"""Toplist after the demodulation: the top_k templates of largest 2F above a
threshold, per work unit, without writing the full 2F array.  Checked
against the GPU's own full 2F output (identical selection, order and values:
the same kernel arithmetic), against the FP64 oracle's toplist (identical
except for templates whose 2F lies within the 2F tolerance of the cut),
and for the edge cases: fewer candidates than top_k, buffer overflow, ties,
batched work units with and without toplists."""
import sys

import numpy as np
import pytest

import oracle
import synth
from synth.device import to_device, alloc_output
from tests._helpers import small_workload, replace, twoF_error

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plan(ws, **kw):
    import paper_0904_1826_amd as P
    return P.Plan(max_sft=max(w.n_sft for w in ws), max_bins=max(w.n_bins for w in ws),
                  max_sky=max(w.n_sky for w in ws), max_fd=max(w.n_fd for w in ws), max_f=max(w.n_f for w in ws),
                  max_dterms=max(max(w.dterms for w in ws), 16), **kw)


def _full_and_top(torch, w, top_k, threshold, **kw):
    """2F of every template (one call) and the toplist alone (another call)."""
    import paper_0904_1826_amd as P
    wu, _ = to_device(w)
    full = alloc_output(w)
    only = alloc_output(w, top_k=top_k, threshold=threshold, full=False)
    with _plan([w], **kw) as p:
        p.compute(wu, full)
        p.compute(wu, only)
        torch.cuda.synchronize()
    return full.twoF.cpu().numpy().ravel(), P.toplist(only)


def _workload(seed=900, **kw):
    args = dict(n_det=2, slots=24, keep=0.85, n_sky=4, n_fd=5, n_f=700, dterms=8,
                injections=((1, 2, 333, 14.0), (3, 4, 100, 9.0), (0, 0, 650, 11.0)))
    args.update(kw)
    return small_workload(seed, **args)


@pytest.mark.parametrize("form", ["interp", "direct", "interp-coef16"])
def test_toplist_equals_selection_of_own_output(torch_cuda, form):
    w = _workload()
    kernel, _, extra = form.partition("-")
    kw = dict(kernel=kernel, coef="f16" if extra == "coef16" else "f32")
    full, (tf, s, i, j, n_above) = _full_and_top(torch_cuda, w, 50, 8.0, **kw)
    idx, n = oracle.toplist(full.astype(np.float64), 8.0, 50)
    _say(f"{form}: n_above {n_above} (full output: {n}), top 2F {tf[:3]}")
    assert n_above == n
    got = (s.astype(np.int64) * w.n_fd + i) * w.n_f + j
    assert np.array_equal(got, idx)
    assert np.array_equal(tf, full[idx].astype(np.float32))        # the very values of the full output


def test_toplist_against_oracle(torch_cuda):
    w = _workload(901)
    top_k, thr = 40, 6.0
    full, (tf, s, i, j, n_above) = _full_and_top(torch_cuda, w, top_k, thr)
    ref = oracle.fstat(w)["twoF"]                                     # linear template order
    ridx, rn = oracle.toplist(ref, thr, top_k)
    got = (s.astype(np.int64) * w.n_fd + i) * w.n_f + j
    e = twoF_error(tf, ref[got])
    assert e.max() <= 1e-4
    # membership may differ only where the 2F is within the tolerance of the cut
    cut = ref[ridx[-1]]
    tol = 1e-4 * max(cut, 4.0)
    for t in set(got) ^ set(ridx):
        assert abs(ref[t] - cut) <= 2 * tol, (t, ref[t], cut)
    near = np.sum(np.abs(ref - thr) <= 1e-4 * max(thr, 4.0))
    assert abs(n_above - rn) <= near
    for x in w.injections:                                           # the injections are found
        assert (x.sky_index * w.n_fd + x.fdot_index) * w.n_f + x.f_index in set(got)


def test_toplist_fewer_candidates_than_k(torch_cuda):
    import paper_0904_1826_amd as P
    w = _workload(902)
    wu, _ = to_device(w)
    out = alloc_output(w, top_k=100, threshold=60.0, full=False)
    with _plan([w]) as p:
        p.compute(wu, out)
        torch_cuda.cuda.synchronize()
    raw = out.top.cpu().numpy()
    tf, s, i, j, n_above = P.toplist(out)
    _say(f"threshold 60: n_above {n_above}")
    assert 0 < n_above < 100
    assert np.all(raw[n_above:, 1:] == -1)
    assert np.all(tf >= 60.0) and np.all(np.diff(tf) <= 0)


def test_toplist_overflow_is_reported(torch_cuda):
    import paper_0904_1826_amd as P
    w = _workload(903)
    wu, _ = to_device(w)
    out = alloc_output(w, top_k=16, threshold=0.0, full=False)        # every template qualifies
    with _plan([w], max_cands=64) as p:
        p.compute(wu, out)
        torch_cuda.cuda.synchronize()
    tf, s, i, j, n_above = P.toplist(out)
    assert n_above == w.n_templates > 64                              # the count keeps going
    assert len(tf) == 16 and np.all(np.diff(tf) <= 0)
    with pytest.raises(P.FstatError) as e:                            # top_k beyond the capacity
        with _plan([w], max_cands=64) as p:
            p.compute(wu, alloc_output(w, top_k=65, threshold=0.0, full=False))
    assert e.value.code == P.FSTAT_E_SIZE


def test_toplist_ties_by_template_index(torch_cuda):
    """Two identical sky points give equal 2F on both: the lower template
    index comes first."""
    w = _workload(904, n_sky=3, injections=((1, 2, 333, 14.0), (0, 4, 100, 9.0)))
    sky = w.sky.copy()
    sky[2] = sky[0]
    w = replace(w, sky=sky, a=np.concatenate([w.a[:2], w.a[:1]]), b=np.concatenate([w.b[:2], w.b[:1]]))
    full, (tf, s, i, j, n_above) = _full_and_top(torch_cuda, w, 30, 6.0)
    per = w.n_fd * w.n_f
    assert np.array_equal(full[:per], full[2 * per:])                # the two copies agree exactly
    got = (s.astype(np.int64) * w.n_fd + i) * w.n_f + j
    idx, _ = oracle.toplist(full.astype(np.float64), 6.0, 30)
    assert np.array_equal(got, idx)
    pairs = [(a, b) for a in range(len(got)) for b in range(len(got)) if got[b] == got[a] + 2 * per]
    assert pairs and all(a < b for a, b in pairs)


def test_batch_toplists_match_single_units(torch_cuda):
    import paper_0904_1826_amd as P
    torch = torch_cuda
    ws = synth.make_batch(3, n_wu=5, scale=0.1)
    devs = [to_device(w)[0] for w in ws]
    # threshold high enough that no unit overflows the default 65536 candidates
    outs = [alloc_output(w, top_k=0 if k == 2 else 25, threshold=14.0, full=(k % 2 == 0)) for k, w in enumerate(ws)]
    with _plan(ws) as p:
        p.batch_compute(devs, outs)
        torch.cuda.synchronize()
        p.batch_compute(devs, outs)                                  # graph replay
        torch.cuda.synchronize()
    for k, w in enumerate(ws):
        if outs[k].top_k == 0:
            continue
        single = alloc_output(w, top_k=25, threshold=14.0, full=False)
        with _plan([w]) as p:
            p.compute(devs[k], single)
            torch.cuda.synchronize()
        a, b = P.toplist(outs[k]), P.toplist(single)
        _say(f"unit {k}: n_above {a[4]} / {b[4]}; batch {a[0][:4]} {a[1][:4]} {a[2][:4]} {a[3][:4]}; "
             f"single {b[0][:4]} {b[1][:4]} {b[2][:4]} {b[3][:4]}")
        assert a[4] == b[4] <= 65536
        for x, y in zip(a[:4], b[:4]):
            assert np.array_equal(x, y)


def test_toplist_work_unit_shaped_case(torch_cuda):
    """The full-size work unit in the benchmark's configuration: the top
    1000 above 2F = 20 without the 5.76e7-template 2F array."""
    import paper_0904_1826_amd as P
    torch = torch_cuda
    w = synth.make_config(1)
    full, (tf, s, i, j, n_above) = _full_and_top(torch, w, 1000, 20.0)
    idx, n = oracle.toplist(full.astype(np.float64), 20.0, 1000)
    _say(f"work unit: n_above {n_above}, top 2F {tf[:4]}")
    assert n_above == n
    got = (s.astype(np.int64) * w.n_fd + i) * w.n_f + j
    assert np.array_equal(got, idx)
    for x in w.injections:
        assert (x.sky_index * w.n_fd + x.fdot_index) * w.n_f + x.f_index in set(got)


def test_batch_graphs_follow_reallocated_toplist_buffers(torch_cuda):
    """Batched calls on one plan of 8 units without toplists, 4 with, 8 with
    (which grows the toplist buffers), and the same 4 again: the last call has
    the shapes of the second, and must not replay the second's graph, which
    holds the old buffers' addresses.  Its toplists equal the second call's
    and the single-unit calls'."""
    import paper_0904_1826_amd as P
    torch = torch_cuda
    ws = [_workload(910 + k, n_sky=2, n_fd=3, n_f=300, injections=((1, 2, 150, 14.0),)) for k in range(8)]
    devs = [to_device(w)[0] for w in ws]
    tops = lambda sel: [alloc_output(ws[k], top_k=20, threshold=8.0, full=False) for k in sel]
    with _plan(ws) as p:
        p.batch_compute(devs, [alloc_output(w) for w in ws])
        second = tops(range(4))
        p.batch_compute(devs[:4], second)
        p.batch_compute(devs, tops(range(8)))
        fourth = tops(range(4))
        p.batch_compute(devs[:4], fourth)
        torch.cuda.synchronize()
    for k in range(4):
        single = alloc_output(ws[k], top_k=20, threshold=8.0, full=False)
        with _plan([ws[k]]) as p:
            p.compute(devs[k], single)
            torch.cuda.synchronize()
        a, b, c = P.toplist(second[k]), P.toplist(fourth[k]), P.toplist(single)
        _say(f"unit {k}: n_above {a[4]} / {b[4]} / {c[4]}")
        assert a[4] == b[4] == c[4] > 0
        for x, y, z in zip(a[:4], b[:4], c[:4]):
            assert np.array_equal(x, y) and np.array_equal(x, z)
