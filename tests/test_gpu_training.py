"""T5-DNN trained on the GPU path's own features (synthetic truth), then
loaded into the library: its scores agree with the FP64 oracle running the
same trained weights, and at the working point matched to the pre-DNN
real-T5 efficiency it keeps fewer fake T5s than the circle-fit chi2 cut."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_13166_amd import train as TR
from paper_2403_13166_amd.synth import events as E, geometry as G, model as M
from tests import compare as CMP

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_trained_model_on_gpu():
    from paper_2403_13166_amd import binding as B
    from paper_2403_13166_amd.runtime import Builder, to_device
    geo = G.make_geometry(True)
    b = Builder(geo.to_blob(), M.make_model().to_blob(), 0)
    try:
        evs = [E.make_event(geo, E.PU200, (5, e)) for e in range(4)]
        X, y, trk, c2, _ = TR.collect(b, evs)
    finally:
        b.close()
    _say(f"training set: {len(y)} T5s, {y.mean():.3f} real")
    res = TR.fit(X, y, epochs=8)
    te = res.test_index
    cmp = TR.compare_selections(TR.predict(res.model, X[te]), c2[te], y[te], trk[te], np.unique(trk[te][y[te]]),
                                geo.params["chi2_rphi_max"])
    _say("held-out rows:", cmp)
    assert cmp["dnn"]["fakes_kept"] < cmp["pre_dnn"]["fakes_kept"]
    # the trained blob in the library against the oracle with the same blob
    ev = E.make_event(geo, E.PU200, (5, 2000))
    og, om = O.Geom(geo.to_blob()), O.Model(res.model.to_blob())
    orc = O.build_objects(og, om, ev.x, ev.y, ev.z, ev.sensor)
    b = Builder(geo.to_blob(), res.model.to_blob(), 0)
    try:
        for prec, tol in ((B.LST_PREC_F32, 1e-5), (B.LST_PREC_BF16, 2e-2)):
            gh = b.build(*to_device(ev, b.device), precision=prec).to_host()
            reps = CMP.compare(og, om, ev, gh, orc)
            assert all(r.violation == 0 for r in reps)
            err = CMP.score_errors(gh, orc)
            _say(f"trained model, precision {prec}: score error {err['score']}")
            assert err["score"][0] <= tol and err["n_common"] > 10_000
    finally:
        b.close()
