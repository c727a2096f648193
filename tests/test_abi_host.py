"""The C ABI on the host: the library loads, exports every declared function,
and validates arguments without touching a GPU."""
import ctypes
import os

import pytest

from paper_1803_00005_amd import hgf

pytestmark = pytest.mark.skipif(not os.path.exists(hgf.LIB_PATH),
                                reason="libhgf.so not built (run __graft_entry__.build())")


def test_library_exports_every_declared_function():
    lib = hgf.lib()
    names = hgf.header_functions()
    assert "hgf_filter" in names and "hgf_guide_filter" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in hgf.h but not exported"


def test_num_channels():
    assert hgf.num_channels(3, 1) == 3
    assert hgf.num_channels(3, 2) == 9
    assert hgf.num_channels(3, 3) == 19
    assert hgf.num_channels(3, 2, "power") == 6
    assert hgf.num_channels(1, 5, "power") == 5
    assert hgf.lib().hgf_num_channels(0, 1, 0) == -1
    assert hgf.lib().hgf_num_channels(3, 1, 7) == -1


def test_supported_set():
    # every channel count 1..19 (e.g. the power basis of RGB at d = 4, n = 12)
    # and every radius 0..9, in both forms
    for n in range(1, 20):
        for r in range(0, 10):
            assert hgf.is_supported(n, r)
            assert hgf.is_supported(n, r, "ridge")
    assert not hgf.is_supported(20, 4)
    assert not hgf.is_supported(0, 4)
    assert not hgf.is_supported(3, 10)
    assert hgf.workspace_size(_p(degree=4, basis="power")) > 0   # n = 12


def _p(**kw):
    base = dict(height=8, width=9, labels=4, radius=2, eps=1e-3, degree=2)
    base.update(kw)
    return hgf.make_params(base.pop("height"), base.pop("width"), base.pop("labels"), **base)


def test_workspace_size_valid():
    ws = hgf.workspace_size(_p())
    assert ws > 0 and ws % 256 == 0
    # more labels never need less workspace
    assert hgf.workspace_size(_p(labels=200)) >= ws


@pytest.mark.parametrize("bad,status", [
    (dict(eps=0.0), hgf.HGF_E_INVALID),
    (dict(eps=-1.0), hgf.HGF_E_INVALID),
    (dict(eps=float("nan")), hgf.HGF_E_INVALID),
    (dict(height=0), hgf.HGF_E_INVALID),
    (dict(width=-3), hgf.HGF_E_INVALID),
    (dict(labels=0), hgf.HGF_E_INVALID),
    (dict(radius=-1), hgf.HGF_E_INVALID),
    (dict(degree=0), hgf.HGF_E_INVALID),
    (dict(guide_channels=4), hgf.HGF_E_INVALID),
    (dict(radius=10), hgf.HGF_E_UNSUPPORTED),
    (dict(degree=4), hgf.HGF_E_UNSUPPORTED),       # n = 34
    (dict(reg="ridge", cost_dtype="bf16"), hgf.HGF_E_UNSUPPORTED),
    (dict(reg="ridge", cost_dtype="f16"), hgf.HGF_E_UNSUPPORTED),
])
def test_workspace_size_rejects(bad, status):
    with pytest.raises(hgf.HGFError) as ei:
        hgf.workspace_size(_p(**bad))
    assert ei.value.status == status
    # a call without a context leaves its detail in the thread's string
    assert hgf.lib().hgf_last_error(None)


def test_null_pointer_arguments():
    lib = hgf.lib()
    assert lib.hgf_workspace_size(None, None) == hgf.HGF_E_INVALID
    p = _p()
    assert lib.hgf_workspace_size(ctypes.byref(p), None) == hgf.HGF_E_INVALID
    assert lib.hgf_filter(None, ctypes.byref(p), None, None, None, None, None, 0, None) == hgf.HGF_E_INVALID
    assert lib.hgf_spd_inverse(None, None, 3, 1, None) == hgf.HGF_E_INVALID
    assert lib.hgf_box_sum(None, None, 1, 1, 1, 0, None) == hgf.HGF_E_INVALID
    assert lib.hgf_guide_filter(None, None, None, 0, 1, 0, None, None, None, None) == hgf.HGF_E_INVALID
    assert lib.hgf_status_string(hgf.HGF_E_UNSUPPORTED) == b"HGF_E_UNSUPPORTED"


@pytest.mark.parametrize("field,value", [("stats_dtype", 1), ("stats_dtype", 2),
                                         ("stats_dtype", -1), ("cost_dtype", 3),
                                         ("cost_dtype", 7)])
def test_dtype_fields_validated(field, value):
    p = _p()
    setattr(p, field, value)
    with pytest.raises(hgf.HGFError) as ei:
        hgf.workspace_size(p)
    assert ei.value.status == hgf.HGF_E_INVALID


def test_float64_solve_records_need_more_workspace():
    # the float64 solve keeps float64 window means and inverses per pixel
    assert hgf.workspace_size(_p(stats_dtype="f64")) > hgf.workspace_size(_p())
    assert hgf.workspace_size(_p(cost_dtype="f16")) == hgf.workspace_size(_p())


def test_ld_smaller_than_labels_rejected():
    with pytest.raises(hgf.HGFError):
        hgf.workspace_size(_p(cost_ld=2))


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message
    before anything touches a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    proc = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2",
                           "--steps", "1", "--warmup", "0"],
                          capture_output=True, text=True, timeout=300, cwd=root)
    assert proc.returncode == 2
    assert "one GPU" in proc.stderr
    assert proc.stdout.strip() == ""
