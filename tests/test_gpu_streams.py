"""Event-level concurrency on one GPU, the analogue of the paper's throughput
at several CUDA streams (Sec. 3): builders with their own contexts, HIP
streams and captured graphs replay their batches at the same time, and on
every replay each builder's objects equal its own eager build bit for bit.

Each builder keeps its input tensors referenced while its graph exists: a
captured graph holds their device addresses.
"""
import sys

import numpy as np
import pytest

from paper_2403_13166_amd.synth import events as E, geometry as G, model as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEYS = ("md_hits", "ls_md", "t3_ls", "t5_t3", "t5_score", "t5_chi2_rphi", "t5_chi2_rz", "event_offsets")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_concurrent_builders_replay_equal_eager():
    from paper_2403_13166_amd import binding as B
    from paper_2403_13166_amd.runtime import Builder
    geo = G.make_geometry(True)
    mdl = M.make_model()
    units = []
    for i in range(3):
        rng = E.event_rng(3, i)
        evs = [E.make_event(geo, E.batch_event_config(rng), (3, i, e)) for e in range(4 + 2 * i)]
        x, y, z, s, off = E.concat_events(evs)
        b = Builder(geo.to_blob(), mdl.to_blob(), 0)
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(b.device)
        d = (T(x), T(y), T(z), T(s), T(off))
        eager = b.build(*d[:4], event_offsets=d[4], precision=B.LST_PREC_BF16).to_host()
        st = torch.cuda.Stream(device=b.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(st):
            b.launch(*d[:4], event_offsets=d[4], precision=B.LST_PREC_BF16)
            st.synchronize()
            with torch.cuda.graph(g, stream=st, capture_error_mode="relaxed"):
                b.launch(*d[:4], event_offsets=d[4], precision=B.LST_PREC_BF16)
        st.synchronize()
        units.append((b, st, g, d, eager))
        _say(f"builder {i}: {len(evs)} events, {len(x)} hits, objects MD/LS/T3/T5 "
             f"{[len(eager.md_hits), len(eager.ls_md), len(eager.t3_ls), len(eager.t5_t3)]}")
    for rep in range(3):
        # clear the outputs, so that every replay has to write them again
        for b, st, g, d, eager in units:
            o = b.view()
            for t in (o.md_hits, o.ls_md, o.t3_ls, o.t5_t3, o.t5_score):
                t.fill_(-1)
        torch.cuda.synchronize()
        for b, st, g, d, eager in units:
            with torch.cuda.stream(st):
                g.replay()
        torch.cuda.synchronize()
        for i, (b, st, g, d, eager) in enumerate(units):
            got = b.view().to_host()
            for k in KEYS:
                assert np.array_equal(getattr(got, k), getattr(eager, k)), (rep, i, k)
        _say(f"replay {rep}: every builder equals its eager build")
    builders = [u[0] for u in units]
    units.clear()                   # graphs and their inputs first, then the contexts
    for b in builders:
        b.close()
