"""Autotuner of the build's launch shapes on the current GPU and workload.

Knobs (all exposed through lst_set_tuning; none changes a result):
  * bin_split: sensor-id ranges per event in hit binning, each sorted by one
    block in LDS (the module-bin size);
  * tile_per[s]: candidates per thread of each compaction stage's 256-thread
    tile (the LDS tile holds the tile's anchor window); the line-segment and
    T3 stages have no compaction tiles, so tile_per[1] and tile_per[2] are not
    searched;
  * eval_blocks: persistent blocks of the compaction kernels;
  * t3_masks: pass masks the T3 stage keeps per wavefront (wavefronts with
    more candidates go to a second kernel that evaluates the rest again).

Search: coordinate descent. Each knob is timed on the stage window it governs
(HIP events recorded on the build stream around that stage), the others held
at their current best; the median of `reps` eager builds decides. Every build
of the search must produce the same object counts as the first one, which
checks on the fly that a tuning changes speed only.
"""
from __future__ import annotations

import statistics

from . import binding as B

BIN_SPLITS = (1, 96, 128)     # sensor ranges per event (raised to what the geometry needs)
EVAL_BLOCKS = (1024, 2048, 4096, 8192)
T3_MASKS = (2, 4, 8)
# (knob, stage index or None, choices, timing window)
KNOBS = (
    ("bin_split", None, BIN_SPLITS, "bin"),
    ("tile_per", 0, B.TILE_CHOICES[0], "md"),
    ("tile_per", 3, B.TILE_CHOICES[3], "t5"),
    ("tile_per", 4, B.TILE_CHOICES[4], "t5"),
    ("eval_blocks", None, EVAL_BLOCKS, "build"),
    ("t3_masks", None, T3_MASKS, "t3"),
)


def _with(t: dict, knob: str, idx, v) -> dict:
    n = {"bin_split": t["bin_split"], "tile_per": list(t["tile_per"]), "eval_blocks": t["eval_blocks"],
         "t3_masks": t.get("t3_masks", B.T3_MASKS_DEFAULT)}
    if idx is None:
        n[knob] = v
    else:
        n[knob][idx] = v
    return n


def autotune(builder, run, sync, reps: int = 5, log=None) -> tuple[dict, list]:
    """Tune `builder`'s context for the build that `run()` enqueues (eagerly,
    with the builder's reserved capacities); `sync()` waits for it. Leaves the
    best tuning set and returns it with the table of timings."""
    ctx = builder.ctx
    B.lst_set_timing(ctx, True)
    best = B.lst_get_tuning(ctx)
    ref_counts = None

    def measure(t: dict, window: str) -> float:
        nonlocal ref_counts
        B.lst_set_tuning(ctx, t)
        run()
        sync()
        c = builder.device_counts()[:4]
        if ref_counts is None:
            ref_counts = c
        elif c != ref_counts:
            raise RuntimeError(f"tuning {t} changed the object counts {ref_counts} -> {c}")
        vals = []
        for _ in range(reps):
            run()
            sync()
            vals.append(B.lst_stage_times(ctx)[window])
        return statistics.median(vals)

    table = []
    for knob, idx, choices, window in KNOBS:
        cur = best[knob] if idx is None else best[knob][idx]
        res = {}
        for v in sorted(set(choices) | {cur}):
            res[v] = measure(_with(best, knob, idx, v), window)
        pick = min(res, key=res.get)
        if res[pick] < res[cur] * 0.98:       # move only on a clear gain
            best = _with(best, knob, idx, pick)
        name = knob if idx is None else f"{knob}[{idx}]"
        table.append({"knob": name, "window": window, "ms": {str(k): v for k, v in res.items()},
                      "chosen": best[knob] if idx is None else best[knob][idx]})
        if log:
            log(f"autotune {name}: " + ", ".join(f"{k}={v:.4f}" for k, v in res.items())
                + f" -> {table[-1]['chosen']}")
    B.lst_set_tuning(ctx, best)
    return best, table
