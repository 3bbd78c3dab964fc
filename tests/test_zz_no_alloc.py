"""GPU test of lst_build_objects_noalloc, the build entry point that takes no
workspace (its scratch is a static per-GPU array): called through the C ABI,
its objects must equal those of lst_build_objects with a caller workspace,
bit for bit, on two calls in a row (the second on a smaller event, so the
static scratch holds the first call's contents), and capacities beyond the
static scratch must be refused with LST_E_INVAL before any GPU work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _events(geo):
    from paper_2403_13166_amd.synth import events as E
    big = E.make_event(geo, E.pileup_event_config(60.0), (4, 900, 0))
    small = E.make_event(geo, E.pileup_event_config(12.0), (4, 900, 1))
    assert small.n < big.n
    return big, small


def _outputs(caps, dev):
    from paper_2403_13166_amd import binding as B
    i32 = dict(dtype=torch.int32, device=dev)
    f32 = dict(dtype=torch.float32, device=dev)
    # a sentinel fill, so entries the build did not write would show up
    t = dict(md_hits=torch.full((caps.md, 2), -7, **i32), ls_md=torch.full((caps.ls, 2), -7, **i32),
             t3_ls=torch.full((caps.t3, 2), -7, **i32), t5_t3=torch.full((caps.t5, 2), -7, **i32),
             t5_score=torch.full((caps.t5,), -7.0, **f32), t5_chi2_rphi=torch.full((caps.t5,), -7.0, **f32),
             t5_chi2_rz=torch.full((caps.t5,), -7.0, **f32),
             counts=torch.zeros(B.LST_COUNTS_LEN, dtype=torch.int64, device=dev))
    s = B.LstObjects(t["md_hits"].data_ptr(), t["ls_md"].data_ptr(), t["t3_ls"].data_ptr(),
                     t["t5_t3"].data_ptr(), t["t5_score"].data_ptr(), t["t5_chi2_rphi"].data_ptr(),
                     t["t5_chi2_rz"].data_ptr(), None, t["counts"].data_ptr(), 0, 0, 0, 0)
    return t, s


def _host(t, s):
    n = (s.n_md, s.n_ls, s.n_t3, s.n_t5)
    return dict(md_hits=t["md_hits"][:n[0]].cpu().numpy(), ls_md=t["ls_md"][:n[1]].cpu().numpy(),
                t3_ls=t["t3_ls"][:n[2]].cpu().numpy(), t5_t3=t["t5_t3"][:n[3]].cpu().numpy(),
                t5_score=t["t5_score"][:n[3]].cpu().numpy(), t5_chi2_rphi=t["t5_chi2_rphi"][:n[3]].cpu().numpy(),
                t5_chi2_rz=t["t5_chi2_rz"][:n[3]].cpu().numpy(), counts=t["counts"].cpu().numpy())


def test_noalloc_build_equals_workspace_build(geo_full, model):
    from paper_2403_13166_amd import binding as B
    from paper_2403_13166_amd.runtime import Builder, Caps, to_device
    dev = torch.device("cuda", 0)
    b = Builder(geo_full.to_blob(), model.to_blob(), 0)
    limit = B.LST_NOALLOC_SCRATCH_MIB << 20
    stream = torch.cuda.current_stream(dev).cuda_stream
    try:
        evs = _events(geo_full)
        dev_ev = [to_device(e, dev) for e in evs]
        # capacities sized from a sizing build, with headroom, per event
        caps = []
        for x, y, z, s in dev_ev:
            o = b.build(x, y, z, s, precision=B.LST_PREC_BF16)
            c = b.device_counts()
            k = Caps(hits=int(x.shape[0]), events=1, md=int(c[0] * 1.2) + 256, ls=int(c[1] * 1.2) + 256,
                     t3=int(c[2] * 1.2) + 256, t5=int(c[3] * 1.2) + 256, cand=int(c[5] * 1.2) + 4096)
            assert o.counts()[0] > 0
            need = B.lst_workspace_size(b.ctx, k.c())
            print(f"event of {x.shape[0]} hits: caps {k}, workspace {need / 2**20:.1f} MiB "
                  f"(static scratch {B.LST_NOALLOC_SCRATCH_MIB} MiB)", flush=True)
            assert need <= limit
            caps.append(k)
        opts = B.LstOptions(B.LST_MODE_DNN, B.LST_PREC_BF16, float("nan"), 0)
        # two allocation-free calls in a row, the second on the smaller event
        for (x, y, z, s), k, ev in zip(dev_ev, caps, evs):
            hits = B.LstHits(x.data_ptr(), y.data_ptr(), z.data_ptr(), s.data_ptr(), int(x.shape[0]))
            tn, sn = _outputs(k, dev)
            B.lst_build_objects_noalloc(b.ctx, hits, opts, k.c(), sn, stream)
            got = _host(tn, sn)
            tw, sw = _outputs(k, dev)
            ws_bytes = B.lst_workspace_size(b.ctx, k.c())
            ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
            B.lst_build_objects(b.ctx, hits, opts, k.c(), sw, (ws.data_ptr() + 255) & ~255, ws_bytes, stream)
            ref = _host(tw, sw)
            print(f"{ev.n} hits: noalloc counts {(sn.n_md, sn.n_ls, sn.n_t3, sn.n_t5)}, "
                  f"workspace counts {(sw.n_md, sw.n_ls, sw.n_t3, sw.n_t5)}", flush=True)
            assert (sn.n_md, sn.n_ls, sn.n_t3, sn.n_t5) == (sw.n_md, sw.n_ls, sw.n_t3, sw.n_t5)
            assert sn.n_t5 > 0
            for key in ref:
                assert np.array_equal(got[key], ref[key]), key
            del ws
        # capacities whose workspace exceeds the static scratch: refused on the host
        x, y, z, s = dev_ev[1]
        hits = B.LstHits(x.data_ptr(), y.data_ptr(), z.data_ptr(), s.data_ptr(), int(x.shape[0]))
        big = Caps(hits=int(x.shape[0]), events=1, md=1 << 20, ls=1 << 20, t3=1 << 20, t5=1 << 20,
                   cand=limit // 32)
        assert B.lst_workspace_size(b.ctx, big.c()) > limit
        tn, sn = _outputs(Caps(1, 1, 1, 1, 1, 1, 1), dev)
        st = B.lst_build_objects_noalloc(b.ctx, hits, opts, big.c(), sn, stream, check=False)
        assert st == B.LST_E_INVAL
        assert "allocation-free" in B.lst_last_error(b.ctx)
    finally:
        b.close()
