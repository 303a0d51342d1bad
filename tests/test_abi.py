"""The C-ABI library loads and exports every entry point include/fstat.h
declares; host-side argument checks work without a GPU."""
import ctypes
import os
import re

import pytest

import paper_0904_1826_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fstat.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fstat_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        P_build = __import__("paper_0904_1826_amd.build", fromlist=["build"])
        P_build.build()
    return P.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert set(names) == set(P.EXPORTS), names
    for n in names:
        assert hasattr(lib, n), n


def test_header_constants_match_the_binding():
    src = open(os.path.join(ROOT, "include", "fstat.h")).read()
    m = re.search(r"#define\s+FSTAT_LAST_TILE_LEN\s+([0-9]+)", src)
    assert m and int(m.group(1)) == P.LAST_TILE_LEN
    m = re.search(r"#define\s+FSTAT_NOALLOC_SCRATCH_BYTES\s+\(([0-9]+)u\s*<<\s*([0-9]+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == P.NOALLOC_SCRATCH_BYTES


def test_strerror(lib):
    for code in range(0, -7, -1):
        assert P.fstat_strerror(code)
    assert P.fstat_strerror(-99) == "unknown error"


def test_plan_create_rejects_bad_descriptors_before_touching_a_device(lib):
    good = dict(max_sft=10, max_bins=100, max_sky=1, max_fd=1, max_f=10, max_dterms=8)
    for bad in (dict(max_dterms=0), dict(max_dterms=65), dict(max_sft=0), dict(max_f=0), dict(storage=7),
                dict(phase=5), dict(kernel=9)):
        d = dict(good, **bad)
        with pytest.raises(P.FstatError) as e:
            P.fstat_plan_create(**d)
        assert e.value.code == P.FSTAT_E_ARG


def test_null_plan_and_null_arguments(lib):
    assert lib.fstat_compute(None, None, None, None) == P.FSTAT_E_ARG
    assert lib.fstat_batch_compute(None, None, 0, None, None) == P.FSTAT_E_ARG
    assert lib.fstat_bins(None, None, 0, None, None, None, None, None, None, None, None) == P.FSTAT_E_ARG
    assert lib.fstat_autotune(None, None, None, None, None) == P.FSTAT_E_ARG
    assert lib.fstat_last_kernel_ms(None) < 0
    assert lib.fstat_last_tile(None, None) == P.FSTAT_E_ARG
    lib.fstat_plan_destroy(None)
    assert lib.fstat_last_error(None) == b""
    assert lib.fstat_plan_create(None, None) == P.FSTAT_E_ARG
    h = ctypes.c_void_p(1)
    assert lib.fstat_plan_create(ctypes.byref(h), None) == P.FSTAT_E_ARG
    assert not h.value


def test_binding_refuses_host_tensors_and_strided_views():
    """The binding hands the library contiguous device arrays only: a strided
    view is refused first (whatever its device), then a host tensor; None
    passes through for the library to report."""
    import torch
    assert P._ptr(None) is None
    with pytest.raises(ValueError, match="contiguous"):
        P._ptr(torch.zeros(4, 3).t())
    with pytest.raises(ValueError, match="device tensors"):
        P._ptr(torch.zeros(4))


def _host_wu(n_sft=5, n_bins=40, n_sky=2, n_fd=3, n_f=7, storage="c64"):
    """A work unit of CPU tensors with the right element types and counts (the
    array checks look only at dtype and shape)."""
    import torch
    from types import SimpleNamespace
    sft = torch.zeros(n_sft, n_bins, 2, dtype=torch.float32 if storage == "c64" else torch.int16)
    return SimpleNamespace(n_det=1, sft=sft, sft_scale=None if storage == "c64" else torch.ones(n_sft),
                           k_first=100, t_sft=1800.0, t_start=torch.zeros(n_sft, dtype=torch.float64),
                           pos=torch.zeros(n_sft, 3, dtype=torch.float64), vel=torch.zeros(n_sft, 3, dtype=torch.float64),
                           sky=torch.zeros(n_sky, 3, dtype=torch.float64), a=torch.zeros(n_sky, n_sft),
                           b=torch.zeros(n_sky, n_sft), f0=100.0, df=1 / 1800, n_f=n_f, fdot0=0.0, dfdot=0.0,
                           n_fd=n_fd, t_ref=0.0, dterms=8)


def test_array_checks_accept_a_consistent_work_unit():
    import torch
    from types import SimpleNamespace
    for storage in ("c64", "bf16"):
        w = _host_wu(storage=storage)
        P.check_work_unit(w, storage)
        n = 2 * 3 * 7
        P.check_output(w, SimpleNamespace(twoF=torch.zeros(2, 3, 7), fa=torch.zeros(n, 2), fb=None, top_k=0))
        P.check_output(w, SimpleNamespace(twoF=None, top_k=5, top=torch.zeros(5, 4, dtype=torch.int32),
                                          n_above=torch.zeros(1, dtype=torch.int64)))


@pytest.mark.parametrize("field,bad,msg", [
    ("a", ("float64", (2, 5)), "element type"),
    ("b", ("float32", (2, 4)), "elements"),
    ("t_start", ("float32", (5,)), "element type"),
    ("pos", ("float64", (5, 2)), "elements"),
    ("vel", ("float64", (4, 3)), "elements"),
    ("sky", ("float32", (2, 3)), "element type"),
])
def test_array_checks_refuse_mistyped_or_short_inputs(field, bad, msg):
    import torch
    w = _host_wu()
    setattr(w, field, torch.zeros(bad[1], dtype=getattr(torch, bad[0])))
    with pytest.raises(ValueError, match=msg):
        P.check_work_unit(w, "c64")


def test_array_checks_refuse_storage_mismatch_and_bad_outputs():
    import torch
    from types import SimpleNamespace
    w = _host_wu()
    with pytest.raises(ValueError, match="element type"):
        P.check_work_unit(w, "bf16")                    # float32 bins under 16-bit storage
    w16 = _host_wu(storage="bf16")
    w16.sft_scale = None
    P.check_work_unit(w16, "bf16")                  # a missing array is the library's to report
    bad_outputs = [
        (dict(twoF=torch.zeros(2, 3, 6), top_k=0), "elements"),
        (dict(twoF=torch.zeros(42, dtype=torch.float64), top_k=0), "element type"),
        (dict(twoF=torch.zeros(42), fa=torch.zeros(42), top_k=0), "elements"),
        (dict(twoF=None, top_k=5, top=torch.zeros(4, 4, dtype=torch.int32),
              n_above=torch.zeros(1, dtype=torch.int64)), "at least"),
        (dict(twoF=None, top_k=5, top=torch.zeros(5, 4, dtype=torch.int32),
              n_above=torch.zeros(1, dtype=torch.int32)), "element type"),
    ]
    for kw, msg in bad_outputs:
        with pytest.raises(ValueError, match=msg):
            P.check_output(w, SimpleNamespace(**kw))


def test_det_offset_length_is_checked_by_the_binding():
    """det_offset is a host array of n_det + 1 entries copied into the call's
    struct; a wrong length is refused before any call."""
    from types import SimpleNamespace
    fields = dict(n_det=2, n_sft=5, n_bins=40, k_first=1, t_sft=1.0, sft=None, sft_scale=None, t_start=None,
                  pos=None, vel=None, n_sky=2, sky=None, a=None, b=None, f0=1.0, df=1.0, n_f=1, fdot0=0.0, dfdot=0.0,
                  n_fd=1, t_ref=0.0, dterms=1)
    with pytest.raises(ValueError, match="det_offset"):
        P._wu_struct(SimpleNamespace(det_offset=[0, 5], **fields))
    s = P._wu_struct(SimpleNamespace(det_offset=[0, 2, 5], **fields))
    arr = ctypes.cast(s.det_offset, ctypes.POINTER(ctypes.c_int64))
    assert [arr[i] for i in range(3)] == [0, 2, 5] and s.n_det == 2
    assert not P._wu_struct(SimpleNamespace(det_offset=None, **fields)).det_offset


def test_noalloc_entry_point_null_arguments(lib):
    assert lib.fstat_compute_noalloc(None, None, None, None) == P.FSTAT_E_ARG
