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
    lib.fstat_plan_destroy(None)
    assert lib.fstat_last_error(None) == b""
    assert lib.fstat_plan_create(None, None) == P.FSTAT_E_ARG
    h = ctypes.c_void_p(1)
    assert lib.fstat_plan_create(ctypes.byref(h), None) == P.FSTAT_E_ARG
    assert not h.value


def test_binding_refuses_host_tensors():
    """The binding hands the library device addresses only: a host tensor (or
    a strided view of one) is refused before any call, and None passes
    through for the library to report."""
    import torch
    import paper_0904_1826_amd as P
    assert P._ptr(None) is None
    for t in (torch.zeros(4), torch.zeros(4, 3).t()):
        with pytest.raises(ValueError, match="device tensors"):
            P._ptr(t)
