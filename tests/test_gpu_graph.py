"""The LST-built graph of Sec. 4 on the GPU (lst_md_graph, lst_gnn_score,
lst_graph_components) against the FP64 oracle (oracle/graph.py,
oracle/gnn.py), through the C ABI.

* Node features: every MD's seven features within 2e-5 (FP32 vs FP64) of the
  oracle's for the same MD (matched by hit keys); edges equal as sets.
* Components on given scores (seeded inputs, the same on both sides): labels
  equal exactly; an id out of range is reported.
* The whole pipeline (features, BF16 edge classifier, components): an edge
  whose oracle score is within the classifier's tolerance (2e-2) of the
  threshold may go either way, so the GPU's components must join everything
  the oracle's confident edges join and nothing more than its confident plus
  marginal edges join; marginal edges are counted.
"""
import sys

import numpy as np
import pytest

from oracle import gnn as OG, graph as GR
from paper_2403_13166_amd.synth import events as E, geometry as G, gnn as SG, model as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL_SCORE = 2e-2


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    from paper_2403_13166_amd.runtime import Builder, EdgeClassifier
    from oracle import oracle as O
    geo = G.make_geometry(True)
    mdl = M.make_model()
    gm = SG.make_gnn_model()
    b = Builder(geo.to_blob(), mdl.to_blob(), 0)
    c = EdgeClassifier(gm.to_blob(), 0)
    yield geo, b, c, gm, O.Geom(geo.to_blob()), O.Model(mdl.to_blob())
    c.close()
    b.close()


def _partition(labels):
    out = {}
    for v, l in enumerate(labels):
        out.setdefault(int(l), set()).add(v)
    return out


def _event(env, pu, key):
    from oracle import oracle as O
    from paper_2403_13166_amd.runtime import to_device
    geo, b, c, gm, og, om = env
    ev = E.make_event(geo, E.pileup_event_config(pu), key)
    d = to_device(ev, b.device)
    objs = b.build(*d)
    r = O.build_objects(og, om, ev.x, ev.y, ev.z, ev.sensor)
    return ev, d, objs, r


def test_md_graph_matches_oracle(env):
    from paper_2403_13166_amd import binding as B
    geo, b, c, gm, og, om = env
    ev, d, objs, r = _event(env, 20.0, (8, 20, 0))
    n_md, n_ls = objs.counts()[:2]
    feat = torch.empty((n_md, 7), dtype=torch.float32, device=b.device)
    src = torch.empty(n_ls, dtype=torch.int32, device=b.device)
    dst = torch.empty(n_ls, dtype=torch.int32, device=b.device)
    ob = B.LstObjects(objs.md_hits.data_ptr(), objs.ls_md.data_ptr(), None, None, None, None, None, None, None,
                      n_md, n_ls, 0, 0)
    hits = B.LstHits(*(t.data_ptr() for t in d), int(d[0].shape[0]))
    B.lst_md_graph(b.ctx, hits, ob, feat.data_ptr(), src.data_ptr(), dst.data_ptr(),
                   torch.cuda.current_stream(b.device).cuda_stream)
    torch.cuda.synchronize()
    md = objs.md_hits.cpu().numpy()
    F = feat.cpu().numpy()
    s, t = src.cpu().numpy(), dst.cpu().numpy()
    assert np.all(np.diff(t) >= 0)                       # the classifier's layout
    X = GR.md_features(ev.x, ev.y, ev.z, ev.sensor, r.md, geo.kind, geo.layer)
    ref = {tuple(k): X[i] for i, k in enumerate(r.md.tolist())}
    keys = [tuple(k) for k in md.tolist()]
    assert set(keys) == set(ref)
    err = max(float(np.max(np.abs(F[i] - ref[k]))) for i, k in enumerate(keys))
    _say(f"MD graph: {n_md} nodes, {n_ls} edges, max feature error {err:.2e}")
    assert err <= 2e-5
    os_, od = GR.ls_edges(r.ls)
    assert {(keys[a], keys[b_]) for a, b_ in zip(s.tolist(), t.tolist())} == \
        {(tuple(r.md[a]), tuple(r.md[b_])) for a, b_ in zip(os_.tolist(), od.tolist())}


@pytest.mark.parametrize("n,e,seed", [(1, 0, 0), (300, 600, 1), (50_000, 120_000, 2)])
def test_components_exact(env, n, e, seed):
    from paper_2403_13166_amd import binding as B
    geo, b, c, gm, og, om = env
    rng = np.random.default_rng([8, 30, seed])
    src = rng.integers(0, n, e).astype(np.int32)
    dst = np.sort(rng.integers(0, n, e)).astype(np.int32)
    sc = rng.random(e).astype(np.float32)
    T = lambda a: torch.from_numpy(a).to(b.device)
    ts, td, tsc = T(src), T(dst), T(sc)
    lab = torch.empty(n, dtype=torch.int32, device=b.device)
    ntc = torch.zeros(1, dtype=torch.int64, device=b.device)
    wsb = B.lst_graph_components_workspace_size(b.ctx, n)
    ws = torch.empty(wsb + 256, dtype=torch.uint8, device=b.device)
    wp = (ws.data_ptr() + 255) & ~255
    st = torch.cuda.current_stream(b.device).cuda_stream
    B.lst_graph_components(b.ctx, n, ts.data_ptr(), td.data_ptr(), tsc.data_ptr(), e, 0.3, 3, lab.data_ptr(),
                           ntc.data_ptr(), wp, wsb, st)
    ref = GR.components(n, src, dst, sc, np.float32(0.3))
    assert lab.cpu().numpy().tolist() == ref.tolist()
    assert int(ntc.item()) == len(GR.track_candidates(ref, 3))
    _say(f"components n={n} e={e}: {len(set(ref.tolist()))} components, {int(ntc.item())} of >= 3 nodes")
    if e:
        bad = td.clone()
        bad[-1] = n                                      # out of range
        with pytest.raises(B.LstError) as ex:
            B.lst_graph_components(b.ctx, n, ts.data_ptr(), bad.data_ptr(), tsc.data_ptr(), e, 0.3, 3,
                                   lab.data_ptr(), ntc.data_ptr(), wp, wsb, st)
        assert ex.value.status == B.LST_E_INVAL


def test_graph_tcs_pipeline(env):
    from paper_2403_13166_amd.runtime import graph_tcs
    geo, b, c, gm, og, om = env
    ev, d, objs, r = _event(env, 12.0, (8, 21, 0))
    thr = 0.5
    res = graph_tcs(b, c, *d, objs, threshold=thr, min_mds=3)
    torch.cuda.synchronize()
    md = objs.md_hits.cpu().numpy()
    keys = [tuple(k) for k in md.tolist()]
    # oracle, on its own build: features, edges, FP64 classifier with the
    # blob's BF16 weights, components; compared by MD hit keys
    X = GR.md_features(ev.x, ev.y, ev.z, ev.sensor, r.md, geo.kind, geo.layer)
    so, do = GR.ls_edges(r.ls)
    mr = gm.rounded()
    ref = OG.edge_scores(mr.W, mr.b, X, so, do)
    okeys = [tuple(k) for k in r.md.tolist()]
    ref_by = {(okeys[a], okeys[b_]): v for a, b_, v in zip(so.tolist(), do.tolist(), ref.tolist())}
    s, t = res.src.cpu().numpy(), res.dst.cpu().numpy()
    got_by = {(keys[a], keys[b_]): v for a, b_, v in zip(s.tolist(), t.tolist(), res.scores.cpu().numpy().tolist())}
    assert set(got_by) == set(ref_by)
    err = max((abs(got_by[k] - ref_by[k]) for k in ref_by), default=0.0)
    sure = ref >= thr + TOL_SCORE
    maybe = ref >= thr - TOL_SCORE
    lo = GR.components(len(okeys), so, do, sure.astype(float), 0.5)
    hi = GR.components(len(okeys), so, do, maybe.astype(float), 0.5)
    lab = dict(zip(keys, res.labels.cpu().numpy().tolist()))
    # every component of the confident edges lies inside one GPU component,
    # every GPU component inside one component of the confident-or-marginal edges
    for comp in _partition(lo).values():
        assert len({lab[okeys[v]] for v in comp}) == 1
    hi_by = {okeys[v]: int(hi[v]) for v in range(len(okeys))}
    gpu_comp = {}
    for k, l in lab.items():
        gpu_comp.setdefault(l, []).append(k)
    for comp in gpu_comp.values():
        assert len({hi_by[k] for k in comp}) == 1
    n_marg = int(np.count_nonzero(maybe & ~sure))
    _say(f"graph TCs: {len(keys)} MDs, {len(s)} LS edges, score error {err:.2e}, marginal edges {n_marg}, "
         f"TCs (>= 3 MDs) {res.n_tc}")
    assert err <= TOL_SCORE
    ref_tc = len(GR.track_candidates(GR.components(len(okeys), so, do, ref, thr), 3))
    assert abs(res.n_tc - ref_tc) <= n_marg
