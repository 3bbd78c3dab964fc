"""Edge classifier on the GPU (BF16 MFMA, FP32 accumulation and states)
against the FP64 oracle: every edge score within 2e-2 absolute; invalid
graphs are rejected."""
import sys

import numpy as np
import pytest

from oracle import gnn as OG
from paper_2403_13166_amd.synth import gnn as SG

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 2e-2


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def clf():
    from paper_2403_13166_amd.runtime import EdgeClassifier
    m = SG.make_gnn_model()
    c = EdgeClassifier(m.to_blob(), 0)
    yield m, c
    c.close()


def _run(c, g):
    dev = c.device
    x = torch.from_numpy(g.x).to(dev)
    s = torch.from_numpy(g.src).to(dev)
    d = torch.from_numpy(g.dst).to(dev)
    out = c.score(x, s, d)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n,e,seed", [(1000, 4000, 0), (5003, 24_999, 1), (40_000, 200_000, 2)])
def test_gnn_matches_oracle(clf, n, e, seed):
    m, c = clf
    g = SG.make_graph(n, e, window=min(2000, n // 10), seed=(93, seed))
    _say("gnn graph", g.n_nodes, g.n_edges)
    got = _run(c, g)
    mr = m.rounded()
    ref = OG.edge_scores(mr.W, mr.b, g.x, g.src, g.dst)
    err = np.abs(got.astype(np.float64) - ref)
    _say("gnn max err", err.max(), "mean", err.mean())
    assert np.all(np.isfinite(got))
    assert err.max() <= TOL


def test_gnn_full_size_sampled(clf):
    m, c = clf
    g = SG.make_graph()                      # 200k nodes, 1M edges
    got = _run(c, g)
    mr = m.rounded()
    ref = OG.edge_scores(mr.W, mr.b, g.x, g.src, g.dst)
    err = np.abs(got.astype(np.float64) - ref)
    _say("gnn full max err", err.max(), "mean", err.mean())
    assert err.max() <= TOL


def test_gnn_edge_cases(clf):
    from paper_2403_13166_amd import binding as B
    m, c = clf
    # nodes without edges; a node with many incoming edges; self loop
    x = np.random.default_rng(5).standard_normal((50, 7)).astype(np.float32)
    src = np.array([1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26,
                    27, 28, 29, 30, 31, 32, 33, 34, 35, 36, 37, 38, 39, 40, 7], np.int32)
    dst = np.array([0] * 40 + [7], np.int32)
    g = SG.Graph(x, src, dst)
    got = _run(c, g)
    mr = m.rounded()
    ref = OG.edge_scores(mr.W, mr.b, x, src, dst)
    assert np.abs(got - ref).max() <= TOL
    # no edges
    dev = c.device
    out = c.score(torch.from_numpy(x).to(dev), torch.zeros(0, dtype=torch.int32, device=dev),
                  torch.zeros(0, dtype=torch.int32, device=dev))
    assert out.shape == (0,)
    # invalid: id out of range, unsorted dst
    for s_bad, d_bad in ((np.array([0, 50], np.int32), np.array([1, 2], np.int32)),
                         (np.array([0, 1], np.int32), np.array([3, 2], np.int32))):
        with pytest.raises(B.LstError) as ei:
            c.score(torch.from_numpy(x).to(dev), torch.from_numpy(s_bad).to(dev), torch.from_numpy(d_bad).to(dev))
        assert ei.value.status == B.LST_E_INVAL
