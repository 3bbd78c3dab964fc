"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers under tests/sanitize/ are built with -fsanitize=address,undefined
and run as subprocesses:
  * blob_fuzz: the library's blob parsers (paper_2403_13166_amd/csrc/
    lst_host.cpp, plain C++ shared with the HIP library) on valid geometry,
    model and edge-classifier blobs and on thousands of mutated copies
    (truncated, extended, bytes, header counts, map entries and doubles
    overwritten); every call must succeed or report an error, and a valid
    blob must be accepted;
  * oracle_fuzz: the FP64 oracle on a seeded event (its counts must equal the
    oracle library's), then on mutated geometry and model blobs (those that
    still load are used for a build) and on hits with an out-of-range sensor.
Any sanitizer report aborts the driver with a nonzero status.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _have(tool):
    return shutil.which(tool) is not None


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    if not (_have("g++") and _have("gcc")):
        pytest.skip("no host compiler")
    d = tmp_path_factory.mktemp("san")
    csrc = os.path.join(ROOT, "paper_2403_13166_amd", "csrc")
    blob = str(d / "blob_fuzz")
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", csrc, os.path.join(ROOT, "tests", "sanitize", "blob_fuzz.cpp"),
                    os.path.join(csrc, "lst_host.cpp"), "-o", blob], check=True)
    orc = str(d / "oracle_fuzz")
    subprocess.run(["gcc", "-std=c99", *SAN, "-ffp-contract=off", os.path.join(ROOT, "tests", "sanitize", "oracle_fuzz.c"),
                    os.path.join(ROOT, "oracle", "lst_oracle.c"), "-lm", "-o", orc], check=True)
    return d, blob, orc


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    return r.stdout


def test_blob_parsers_under_sanitizers(drivers, geo_barrel, geo_full, model):
    from paper_2403_13166_amd.synth import gnn as SG
    d, blob, _ = drivers
    cases = [("geom", geo_barrel.to_blob(), 3000), ("geom", geo_full.to_blob(), 300),
             ("model", model.to_blob(), 3000), ("gnn", SG.make_gnn_model().to_blob(), 2000)]
    for i, (kind, data, n) in enumerate(cases):
        p = d / f"{kind}{i}.bin"
        p.write_bytes(data)
        out = _run([blob, kind, str(p), str(11 + i), str(n)])
        # the mutations are not all rejected, nor all accepted
        acc = int(out.split("accepted")[0].split(",")[-1])
        rej = int(out.split("rejected")[0].split(",")[-1].split()[0])
        assert acc + rej == n and rej > n // 4, out


def test_oracle_under_sanitizers(drivers, geo_barrel, model):
    from oracle import oracle as O
    from paper_2403_13166_amd.synth import events as E
    d, _, orc = drivers
    ev = E.make_event(geo_barrel, E.SMALL_BARREL, (0, 3))
    (d / "g.bin").write_bytes(geo_barrel.to_blob())
    (d / "m.bin").write_bytes(model.to_blob())
    (d / "h.bin").write_bytes(struct.pack("<q", ev.n) + ev.x.tobytes() + ev.y.tobytes() + ev.z.tobytes()
                              + ev.sensor.astype(np.int32).tobytes())
    out = _run([orc, "fuzz", str(d / "g.bin"), str(d / "m.bin"), str(d / "h.bin"), "7", "400"])
    counts = tuple(int(v) for v in out.split("counts")[1].split("\n")[0].split())
    ref = O.build_objects(O.Geom(geo_barrel.to_blob()), O.Model(model.to_blob()), ev.x, ev.y, ev.z, ev.sensor)
    assert counts == ref.counts() and counts[3] > 0
    assert "fuzz: 400 geometry mutations" in out
