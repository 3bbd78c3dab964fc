"""Host logic on the CPU: capacity growth, the autotuner's search (against a
fake context), the tuning struct, and the benchmark's single-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_caps_growth_covers_counts_and_is_bounded():
    from paper_2403_13166_amd.runtime import Caps
    c = Caps(hits=1000, events=1, md=100, ls=100, t3=100, t5=100, cand=1000)
    # MD overflowed by 3x: later stages saw a truncated input, so they are scaled up (bounded)
    g = c.grown([300, 250, 400, 90, 0, 5000, 0, 0])
    assert g.md >= 300 and g.ls >= 250 * 3 and g.t3 >= 400 * 3 and g.t5 >= 100
    assert g.cand >= 5000
    assert g.hits == c.hits and g.events == c.events
    huge = c.grown([10 ** 6, 10 ** 6, 10 ** 6, 10 ** 6, 0, 10 ** 7, 0, 0])
    assert huge.t3 <= int(10 ** 6 * 8 * 1.25) + 1024        # truncation factor capped at 8
    same = c.grown([10, 10, 10, 10, 0, 10, 0, 0])      # never shrinks
    assert all(getattr(same, k) >= getattr(c, k) for k in ("md", "ls", "t3", "t5", "cand"))


def test_tuning_struct_roundtrip():
    from paper_2403_13166_amd import binding as B
    d = {"bin_split": 8, "tile_per": [2, 8, 4, 1, 2], "eval_blocks": 2048, "t3_masks": 3}
    assert B.LstTuning.from_dict(d).as_dict() == d
    d.pop("t3_masks")                                   # optional: the default
    assert B.LstTuning.from_dict(d).as_dict()["t3_masks"] == B.T3_MASKS_DEFAULT


def test_autotune_search_with_fake_context(monkeypatch):
    from paper_2403_13166_amd import autotune as AT
    from paper_2403_13166_amd import binding as B
    state = {"tuning": {"bin_split": 4, "tile_per": [4, 4, 2, 2, 1], "eval_blocks": 4096, "t3_masks": 8},
             "timing": False}

    def fake_times(ctx):
        t = state["tuning"]
        # T5 pre-cuts fastest at 4, binning fastest at 128, eval grid fastest at 2048; others flat
        return {"build": 1.0 + abs(t["eval_blocks"] - 2048) / 8192, "bin": 0.5 - 0.001 * t["bin_split"],
                "md": 0.1, "ls": 1.0, "t3": 0.05 + 0.01 * (t["t3_masks"] == 2), "t5": 1.0 / t["tile_per"][3],
                "score": 0.2}

    monkeypatch.setattr(B, "lst_set_timing", lambda ctx, on: state.update(timing=on))
    monkeypatch.setattr(B, "lst_get_tuning", lambda ctx: {k: (list(v) if isinstance(v, list) else v)
                                                          for k, v in state["tuning"].items()})
    monkeypatch.setattr(B, "lst_set_tuning", lambda ctx, t: state.update(tuning=t))
    monkeypatch.setattr(B, "lst_stage_times", fake_times)

    class FakeBuilder:
        ctx = object()

        def device_counts(self):
            return [10, 20, 30, 40, 0, 0, 0, 0]

    best, table = AT.autotune(FakeBuilder(), lambda: None, lambda: None, reps=1)
    assert best["tile_per"][3] == 4 and best["bin_split"] == 128 and best["eval_blocks"] == 2048
    assert best["tile_per"][0] == 4                     # flat timings: no move without a clear gain
    assert best["tile_per"][1] == 4                     # the line-segment stage has no tiles: not searched
    assert best["tile_per"][2] == 2 and best["t3_masks"] == 8   # nor the T3 stage; masks: no clear gain
    assert len(table) == len(AT.KNOBS) and state["tuning"] == best

    class ChangingBuilder(FakeBuilder):
        n = 0

        def device_counts(self):
            self.n += 1
            return [10, 20, 30, 40 + (self.n > 1), 0, 0, 0, 0]

    with pytest.raises(RuntimeError):
        AT.autotune(ChangingBuilder(), lambda: None, lambda: None, reps=1)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
