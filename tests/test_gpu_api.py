"""Error behaviour of the C ABI (statuses and messages), through the binding."""
import ctypes as C

import numpy as np
import pytest

from paper_2403_13166_amd.synth import geometry as G, gnn as SG, model as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_api_errors():
    from paper_2403_13166_amd import binding as B
    L = B.lib()
    ctx = B.lst_create(0)
    try:
        geo = G.make_geometry(False).to_blob()
        mdl = M.make_model().to_blob()
        # nothing loaded yet
        caps = B.LstCaps(100, 1, 100, 100, 100, 100, 1000)
        n = C.c_size_t()
        assert L.lst_workspace_size(ctx, C.byref(caps), C.byref(n)) in (B.LST_OK, B.LST_E_STATE)
        X = torch.zeros((4, 42), dtype=torch.float32, device="cuda")
        out = torch.zeros(4, dtype=torch.float32, device="cuda")
        assert L.lst_score(ctx, X.data_ptr(), 0, 4, out.data_ptr(), 0, None) == B.LST_E_STATE
        assert "model" in B.lst_last_error(ctx)
        # malformed blobs
        for blob in (geo[:100], b"XXXX" + geo[4:], geo + b"\0"):
            assert L.lst_load_geometry(ctx, blob, len(blob)) == B.LST_E_INVAL
        for blob in (mdl[:50], b"XXXX" + mdl[4:], mdl + b"\0\0\0\0"):
            assert L.lst_load_model(ctx, blob, len(blob)) == B.LST_E_INVAL
        g = SG.make_gnn_model().to_blob()
        for blob in (g[:30], b"XXXX" + g[4:], g[:-4]):
            assert L.lst_load_gnn(ctx, blob, len(blob)) == B.LST_E_INVAL
        assert L.lst_gnn_score(ctx, None, 0, None, None, 0, None, None, 0, 0, None) == B.LST_E_STATE
        # loaded: argument errors
        B.lst_load_geometry(ctx, geo)
        B.lst_load_model(ctx, mdl)
        assert L.lst_score(ctx, X.data_ptr(), 7, 4, out.data_ptr(), 0, None) == B.LST_E_INVAL
        assert L.lst_score(ctx, X.data_ptr(), 0, 4, out.data_ptr(), 9, None) == B.LST_E_INVAL
        assert L.lst_score(ctx, None, 0, 4, out.data_ptr(), 0, None) == B.LST_E_INVAL
        assert L.lst_score(ctx, X.data_ptr(), 0, 0, out.data_ptr(), 0, None) == B.LST_OK
        ws_bytes = B.lst_workspace_size(ctx, caps)
        ws = torch.empty(ws_bytes + 512, dtype=torch.uint8, device="cuda")
        base = (ws.data_ptr() + 255) & ~255
        x = torch.zeros(10, dtype=torch.float32, device="cuda")
        s = torch.zeros(10, dtype=torch.int32, device="cuda")
        hits = B.LstHits(x.data_ptr(), x.data_ptr(), x.data_ptr(), s.data_ptr(), 10)
        i32 = lambda k: torch.zeros((k, 2), dtype=torch.int32, device="cuda")
        f32 = lambda k: torch.zeros(k, dtype=torch.float32, device="cuda")
        bufs = [i32(100), i32(100), i32(100), i32(100), f32(100), f32(100), f32(100)]
        cnt = torch.zeros(8, dtype=torch.int64, device="cuda")
        objs = B.LstObjects(*[b.data_ptr() for b in bufs], None, cnt.data_ptr(), 0, 0, 0, 0)
        opt = B.LstOptions(0, 0, float("nan"), 0)
        call = lambda o=opt, c=caps, w=base, wb=ws_bytes, h=hits: L.lst_build_objects(
            ctx, C.byref(h), C.byref(o), C.byref(c), C.byref(objs), w, wb, None)
        assert call() == B.LST_OK
        assert call(w=base + 16) == B.LST_E_INVAL                       # misaligned workspace
        assert call(wb=ws_bytes - 1) == B.LST_E_INVAL                   # workspace too small
        assert call(o=B.LstOptions(5, 0, float("nan"), 0)) == B.LST_E_INVAL
        assert call(o=B.LstOptions(0, 3, float("nan"), 0)) == B.LST_E_INVAL
        big = B.LstHits(x.data_ptr(), x.data_ptr(), x.data_ptr(), s.data_ptr(), 1000)
        assert call(h=big) == B.LST_E_INVAL                             # more hits than caps.hits
        assert "caps.hits" in B.lst_last_error(ctx)
        for st in (B.LST_OK, B.LST_E_INVAL, B.LST_E_STATE, B.LST_E_CAPACITY, B.LST_E_HIP, B.LST_E_NOMEM, 42):
            assert isinstance(B.lst_status_string(st), str) and B.lst_status_string(st)
    finally:
        B.lst_destroy(ctx)


def test_failure_injection_per_stage(monkeypatch):
    """Each pipeline stage can be made to fail from the host: the build
    returns LST_E_HIP naming the stage, and the context then builds the same
    objects as before."""
    from paper_2403_13166_amd import binding as B
    from paper_2403_13166_amd.runtime import Builder, to_device
    from paper_2403_13166_amd.synth import events as E
    geo = G.make_geometry(False)
    b = Builder(geo.to_blob(), M.make_model().to_blob(), 0)
    try:
        ev = E.make_event(geo, E.SMALL_BARREL, (0, 1))
        d = to_device(ev, b.device)
        cnt = lambda o: (len(o.md_hits), len(o.ls_md), len(o.t3_ls), len(o.t5_t3))
        ref = b.build(*d).to_host()
        assert cnt(ref)[1] > 0
        for k in range(1, 7):
            print("inject before stage", k, flush=True)
            B.lst_set_fail_stage(b.ctx, k)
            with pytest.raises(B.LstError) as e:
                b.build(*d)
            assert e.value.status == B.LST_E_HIP and f"stage {k}" in str(e.value)
            B.lst_set_fail_stage(b.ctx, 0)
            again = b.build(*d).to_host()
            assert cnt(again) == cnt(ref)
            assert np.array_equal(again.ls_md, ref.ls_md) and np.array_equal(again.t5_t3, ref.t5_t3)
        with pytest.raises(B.LstError) as e:
            B.lst_set_fail_stage(b.ctx, 7)
        assert e.value.status == B.LST_E_INVAL
    finally:
        b.close()
    # the environment switch applies to contexts created while it is set
    monkeypatch.setenv("LST_FAIL_AT_STAGE", "4")
    b2 = Builder(geo.to_blob(), M.make_model().to_blob(), 0)
    monkeypatch.delenv("LST_FAIL_AT_STAGE")
    try:
        with pytest.raises(B.LstError) as e:
            b2.build(*d)
        assert "stage 4" in str(e.value)
        B.lst_set_fail_stage(b2.ctx, 0)
        assert cnt(b2.build(*d).to_host()) == cnt(ref)
    finally:
        b2.close()
