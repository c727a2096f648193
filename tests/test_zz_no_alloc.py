"""hgf_filter_static, the allocation-free entry point (run on an MI355X).

It runs the plain filter with its workspace in the library's static device
array.  Two calls in a row, the second on a smaller input, must each equal
hgf_filter with a caller-given workspace bit for bit (the same kernels, and
a band partition that does not depend on the launch-group size), and an
input whose workspace exceeds the array is refused before anything runs.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1803_00005_amd import hgf, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _lib():
    lib = hgf.lib()
    lib.hgf_filter_static.restype = ctypes.c_int
    lib.hgf_filter_static.argtypes = [ctypes.c_void_p, ctypes.POINTER(hgf.Params)] + \
        [ctypes.c_void_p] * 5
    lib.hgf_static_scratch_bytes.restype = ctypes.c_size_t
    lib.hgf_static_scratch_bytes.argtypes = []
    return lib


def _static(ctx, guide, cost, w):
    lib = _lib()
    p = hgf.make_params(w.height, w.width, w.labels, radius=w.radius, eps=w.eps,
                        degree=w.degree, basis=w.basis)
    Z = torch.empty((w.height, w.width, w.labels), dtype=torch.float32, device="cuda")
    lab = torch.empty((w.height, w.width), dtype=torch.int32, device="cuda")
    st = lib.hgf_filter_static(ctx.handle, ctypes.byref(p), guide.data_ptr(), cost.data_ptr(),
                               Z.data_ptr(), lab.data_ptr(),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, Z, lab


def W(name, **kw):
    base = dict(name=name, height=40, width=50, regions=8, labels=16, radius=4, eps=1e-4,
                degree=1, disparity="planar", seed=7)
    base.update(kw)
    return synth.Workload(**base)


CALLS = [
    # larger first, then smaller: the second call finds the first's contents
    W("static_n9_two_chunks", height=90, width=120, labels=100, radius=9, degree=2, seed=71),
    W("static_rgb64", height=64, width=64, labels=16, radius=4, degree=1, seed=72,
      regions=12, disparity="region_int"),
]


def test_static_entry_point_equals_plain_call():
    ctx = hgf.Context(0)
    for w in CALLS:
        print(f"static call {w.name}: {w.height}x{w.width} n={w.n} L={w.labels}", flush=True)
        g, c = synth.make_workload(w)
        gd = torch.from_numpy(g).cuda()
        cd = torch.from_numpy(c).cuda()
        st, Zs, ls = _static(ctx, gd, cd, w)
        assert st == hgf.HGF_OK, hgf.lib().hgf_last_error(ctx.handle)
        ws = torch.empty(hgf.workspace_size(hgf.make_params(
            w.height, w.width, w.labels, radius=w.radius, eps=w.eps, degree=w.degree)),
            dtype=torch.uint8, device="cuda")
        Zp, lp = ctx.filter(gd, cd, radius=w.radius, eps=w.eps, degree=w.degree, workspace=ws)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(Zs.cpu().numpy(), Zp.cpu().numpy())
        np.testing.assert_array_equal(ls.cpu().numpy(), lp.cpu().numpy())
    ctx.close()


def test_static_entry_point_refuses_oversized_inputs():
    ctx = hgf.Context(0)
    lib = _lib()
    cap = lib.hgf_static_scratch_bytes()
    # about 3 KB of workspace per pixel at n = 19: far more pixels than fit
    w = W("static_too_big", height=1000, width=1000, labels=8, radius=9, degree=3, eps=1e-3)
    p = hgf.make_params(w.height, w.width, w.labels, radius=w.radius, eps=w.eps,
                        degree=w.degree)
    assert hgf.workspace_size(p) > cap
    g = torch.zeros((3, w.height, w.width), dtype=torch.float32, device="cuda")
    c = torch.zeros((w.height, w.width, w.labels), dtype=torch.float32, device="cuda")
    lab = torch.empty((w.height, w.width), dtype=torch.int32, device="cuda")
    st = lib.hgf_filter_static(ctx.handle, ctypes.byref(p), g.data_ptr(), c.data_ptr(),
                               None, lab.data_ptr(), None)
    assert st == hgf.HGF_E_NOMEM
    assert b"static workspace" in lib.hgf_last_error(ctx.handle)
    ctx.close()
