"""The batched and serving forms and the autotuner (run on an MI355X).

Every image of a batch and every request of a served mix must equal the
plain single-image call bit for bit (same kernels, same tuning), and the
plain call is held to the oracle by the parity tests.  The batched form is
replayed from its cached graph several times with the program's own eager
work between replays; each replay is checked.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import hgf_oracle as O  # noqa: E402
from paper_1803_00005_amd import hgf, synth  # noqa: E402

pytestmark = pytest.mark.gpu

REL_TOL = 1e-4
TIE_GAP = 1e-5


def say(msg):
    print(msg, flush=True)


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(dev())
    return t.to(dtype) if dtype is not None else t


def W(name, **kw):
    base = dict(name=name, height=40, width=50, regions=8, labels=16, radius=4, eps=1e-4,
                degree=1, disparity="planar", seed=7)
    base.update(kw)
    return synth.Workload(**base)


MIX = [
    W("mix_a", height=64, width=64, labels=16, radius=4, degree=1, seed=31),
    W("mix_b", height=75, width=130, labels=60, radius=9, degree=2, seed=32),
    W("mix_c", height=33, width=200, labels=70, radius=9, degree=3, eps=1e-3, seed=33),
    W("mix_d", height=90, width=61, labels=64, radius=4, degree=2, seed=34, cost_dtype="bf16"),
    W("mix_e", height=20, width=300, labels=130, radius=9, degree=3, eps=1e-3, seed=35,
      cost_dtype="bf16"),
    W("mix_f", height=1, width=1, labels=3, radius=4, degree=1, seed=36),
]


def inputs(w):
    guide, cost = synth.make_workload(w)
    cdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[w.cost_dtype]
    return guide, cost, to_dev(guide), to_dev(cost, cdt)


@pytest.fixture(scope="module")
def data():
    return [inputs(w) for w in MIX]


@pytest.fixture(scope="module")
def singles(data):
    ctx = hgf.Context(0)
    res = []
    for w, (_, _, g, c) in zip(MIX, data):
        Z, lab = ctx.filter(g, c, radius=w.radius, eps=w.eps, degree=w.degree)
        torch.cuda.synchronize()
        res.append((Z.cpu().numpy(), lab.cpu().numpy()))
    ctx.close()
    return res


def test_singles_match_oracle(data, singles):
    for w, (guide, cost, _, _), (Z, lab) in zip(MIX, data, singles):
        say(f"oracle check {w.name}")
        Zo = O.filter_covariance(O.guidance(guide, w.degree, w.basis), cost, w.radius, w.eps)
        scale = np.maximum(np.abs(Zo), np.abs(cost).max())
        rel = (np.abs(Z - Zo) / scale).max()
        assert rel <= REL_TOL, f"{w.name}: {rel:.3e}"
        ok = (lab == O.wta(Zo)) | O.near_tie_mask(Zo, TIE_GAP)
        assert ok.all()


def _items(data):
    return [dict(guide=g, cost=c, radius=w.radius, eps=w.eps, degree=w.degree)
            for w, (_, _, g, c) in zip(MIX, data)]


def test_batch_graph_replays(data, singles):
    ctx = hgf.Context(0)
    outs = [(torch.empty(w.height, w.width, w.labels, dtype=torch.float32, device=dev()),
             torch.empty(w.height, w.width, dtype=torch.int32, device=dev())) for w in MIX]
    other_g, other_c = data[1][2], data[1][3]
    for rep in range(4):
        say(f"batch replay {rep}")
        # eager work of the program between replays: clear the outputs and run a plain call
        for z, lb in outs:
            z.fill_(float("nan"))
            lb.fill_(-7)
        ctx.filter(other_g, other_c, radius=MIX[1].radius, eps=MIX[1].eps, degree=MIX[1].degree)
        res = ctx.filter_batch(_items(data), outputs=outs)
        torch.cuda.synchronize()
        for w, (z, lb), (Zs, ls) in zip(MIX, res, singles):
            np.testing.assert_array_equal(z.cpu().numpy(), Zs, err_msg=f"{w.name} replay {rep}")
            np.testing.assert_array_equal(lb.cpu().numpy(), ls, err_msg=f"{w.name} replay {rep}")
    # a different output buffer is a different signature: captured afresh
    say("batch with new buffers")
    res = ctx.filter_batch(_items(data))
    torch.cuda.synchronize()
    for w, (z, lb), (Zs, ls) in zip(MIX, res, singles):
        np.testing.assert_array_equal(z.cpu().numpy(), Zs, err_msg=w.name)
        np.testing.assert_array_equal(lb.cpu().numpy(), ls, err_msg=w.name)
    ctx.close()


def test_batch_labels_only_entries(data, singles):
    ctx = hgf.Context(0)
    lib = hgf.lib()
    n = 3
    arr = (hgf.Params * n)()
    import ctypes
    guides = (ctypes.c_void_p * n)()
    costs = (ctypes.c_void_p * n)()
    outs = (ctypes.c_void_p * n)()
    labs = (ctypes.c_void_p * n)()
    keep = []
    for i in range(n):
        w = MIX[i]
        g, c = data[i][2], data[i][3]
        arr[i] = hgf.make_params(w.height, w.width, w.labels, radius=w.radius, eps=w.eps,
                                 degree=w.degree)
        z = torch.empty(w.height, w.width, w.labels, dtype=torch.float32, device=dev())
        lb = torch.empty(w.height, w.width, dtype=torch.int32, device=dev())
        keep.append((z, lb))
        guides[i], costs[i] = g.data_ptr(), c.data_ptr()
        outs[i] = None if i == 1 else z.data_ptr()   # image 1: labels only
        labs[i] = None if i == 2 else lb.data_ptr()  # image 2: filtered costs only
    say("batch with labels-only and out-only entries")
    st = lib.hgf_filter_batch(ctx.handle, n, arr, guides, costs, outs, labs,
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == hgf.HGF_OK, lib.hgf_last_error(ctx.handle)
    torch.cuda.synchronize()
    for i in range(n):
        Zs, ls = singles[i]
        if i != 1:
            np.testing.assert_array_equal(keep[i][0].cpu().numpy(), Zs)
        if i != 2:
            np.testing.assert_array_equal(keep[i][1].cpu().numpy(), ls)
    # an entry with neither output is rejected before anything is enqueued
    outs[0] = None
    labs[0] = None
    st = lib.hgf_filter_batch(ctx.handle, n, arr, guides, costs, outs, labs, None)
    assert st == hgf.HGF_E_INVALID
    assert b"image 0" in lib.hgf_last_error(ctx.handle)
    ctx.close()


def test_autotune_and_table_io(data, tmp_path):
    ctx = hgf.Context(0)
    w = MIX[1]
    _, _, g, c = data[1]
    say("autotune")
    out = torch.empty(w.height, w.width, w.labels, dtype=torch.float32, device=dev())
    ctx.autotune(g, c, radius=w.radius, eps=w.eps, degree=w.degree, out=out)
    rows = ctx.tune_entries()
    assert len(rows) == 3
    assert {r[0] for r in rows} == {0, 1, 2}
    for r in rows:
        assert r[1] == w.n and r[2] == w.radius and r[6] >= 1
    # the tuned path still meets the bar
    guide, cost = data[1][0], data[1][1]
    Zo = O.filter_covariance(O.guidance(guide, w.degree, w.basis), cost, w.radius, w.eps)
    Z, lab = ctx.filter(g, c, radius=w.radius, eps=w.eps, degree=w.degree)
    torch.cuda.synchronize()
    rel = (np.abs(Z.cpu().numpy() - Zo) / np.maximum(np.abs(Zo), np.abs(cost).max())).max()
    assert rel <= REL_TOL
    np.testing.assert_allclose(out.cpu().numpy(), Z.cpu().numpy(), rtol=0, atol=0)
    path = os.path.join(tmp_path, "tune.txt")
    ctx.tune_save(path)
    ctx2 = hgf.Context(0)
    ctx2.tune_load(path)
    assert sorted(ctx2.tune_entries()) == sorted(rows)
    with pytest.raises(hgf.HGFError) as e:
        ctx2.tune_set((7, 1, 1, 0, 0, 1, 10))
    assert e.value.status == hgf.HGF_E_INVALID
    ctx2.close()
    ctx.close()


def _serve(data, slots, arena_bytes, order):
    """Submit the MIX requests in `order` to a fresh server; returns results by index."""
    ctx = hgf.Context(0)
    srv = hgf.Server(ctx, slots=slots, arena_bytes=arena_bytes, max_queue=64)
    res = {}
    ids = {}
    for i in order:
        w = MIX[i]
        g, c = data[i][2], data[i][3]
        z = torch.empty(w.height, w.width, w.labels, dtype=torch.float32, device=dev())
        lb = torch.empty(w.height, w.width, dtype=torch.int32, device=dev())
        ids[srv.submit(g, c, z, lb, radius=w.radius, eps=w.eps, degree=w.degree)] = i
        res[i] = (z, lb)
    srv.drain()
    done = srv.poll(64)
    assert sorted(d.id for d in done) == sorted(ids)
    for d in done:
        assert d.status == hgf.HGF_OK
        assert 0.0 <= d.start_ms <= d.end_ms
    stats = srv.stats()
    assert stats["pending"] == 0 and stats["running"] == 0 and stats["arena_in_use"] == 0
    assert stats["arena_peak"] <= stats["arena_bytes"]
    torch.cuda.synchronize()
    out = {i: (z.cpu().numpy(), lb.cpu().numpy()) for i, (z, lb) in res.items()}
    srv.close()
    ctx.close()
    return out, stats


def test_server_alone_equals_mix(data, singles):
    sizes = [hgf.workspace_size(hgf.make_params(w.height, w.width, w.labels, radius=w.radius,
                                                eps=w.eps, degree=w.degree)) for w in MIX]
    # alone: one request at a time in a one-slot server
    for i in range(len(MIX)):
        say(f"serve alone {MIX[i].name}")
        out, _ = _serve(data, 1, sizes[i] + 4096, [i])
        np.testing.assert_array_equal(out[i][0], singles[i][0])
        np.testing.assert_array_equal(out[i][1], singles[i][1])
    # the mix: every request at once, four slots, an arena that holds only
    # about two of the largest at a time so later requests must queue
    say("serve the mix")
    arena = 2 * max(sizes) + 8192
    out, stats = _serve(data, 4, arena, list(reversed(range(len(MIX)))))
    for i in range(len(MIX)):
        np.testing.assert_array_equal(out[i][0], singles[i][0], err_msg=MIX[i].name)
        np.testing.assert_array_equal(out[i][1], singles[i][1], err_msg=MIX[i].name)
    assert stats["completed"] == len(MIX)


def test_server_admission_errors(data):
    ctx = hgf.Context(0)
    w = MIX[1]
    p = hgf.make_params(w.height, w.width, w.labels, radius=w.radius, eps=w.eps, degree=w.degree)
    need = hgf.workspace_size(p)
    g, c = data[1][2], data[1][3]
    z = torch.empty(w.height, w.width, w.labels, dtype=torch.float32, device=dev())
    lb = torch.empty(w.height, w.width, dtype=torch.int32, device=dev())
    # a request that can never fit
    srv = hgf.Server(ctx, slots=2, arena_bytes=need // 2, max_queue=4)
    with pytest.raises(hgf.HGFError) as e:
        srv.submit(g, c, z, lb, radius=w.radius, eps=w.eps, degree=w.degree)
    assert e.value.status == hgf.HGF_E_NOMEM
    with pytest.raises(hgf.HGFError) as e:
        srv.submit(g, c, z, lb, radius=w.radius, eps=-1.0, degree=w.degree)
    assert e.value.status == hgf.HGF_E_INVALID
    srv.close()
    # a full queue: the submitting stream holds the first request back (a
    # bounded spin kernel), the arena holds one request, the queue one more
    srv = hgf.Server(ctx, slots=1, arena_bytes=need + 4096, max_queue=1)
    side = torch.cuda.Stream()
    z2 = torch.empty_like(z)
    lb2 = torch.empty_like(lb)
    with torch.cuda.stream(side):
        torch.cuda._sleep(20_000_000)
        a = srv.submit(g, c, z, lb, radius=w.radius, eps=w.eps, degree=w.degree, stream=side)
        b = srv.submit(g, c, z2, lb2, radius=w.radius, eps=w.eps, degree=w.degree, stream=side)
        with pytest.raises(hgf.HGFError) as e:
            srv.submit(g, c, z2, lb2, radius=w.radius, eps=w.eps, degree=w.degree, stream=side)
        assert e.value.status == hgf.HGF_E_BUSY
    st = srv.stats()
    assert st["pending"] + st["running"] + st["completed"] == 2
    srv.drain()
    done = srv.poll(8)
    assert sorted(d.id for d in done) == sorted([a, b])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(z.cpu().numpy(), z2.cpu().numpy())
    np.testing.assert_array_equal(lb.cpu().numpy(), lb2.cpu().numpy())
    srv.close()
    ctx.close()
