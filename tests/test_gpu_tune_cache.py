"""The autotuner's choices persist across processes through FWI_TUNE_CACHE.

A tuned forward call appends one line (key : S TZ graph_steps prefetch
prefetch_reverse S_rev TZ_rev reverse_steps forward_steps) to the file.  After fwi_tune_reset (which stands for a
fresh process) the library reads the file back instead of tuning again, and
its results still match the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import tiny_24x16

from helpers import TRACE_TOL, rel, report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NT = 137   # a record length no other test uses, so the tuning key is new


def lines(path):
    with open(path) as f:
        return [ln for ln in f.read().splitlines() if ln.strip()]


def chosen(q):
    return (q["tile_rows"], q["graph_steps"], q["prefetch"], q["prefetch_reverse"])


def test_tuned_choice_round_trips_through_file(tmp_path, monkeypatch):
    cache = str(tmp_path / "tune.txt")
    monkeypatch.setenv("FWI_TUNE_CACHE", cache)
    w = tiny_24x16(nt=NT)
    ref = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    ex = B.make_exec(autotune=1)

    got = B.forward(w.v_true, w.wavelet, w.grid, w.geom, ex).cpu().numpy()
    assert report("forward tiny autotuned (tunes)", rel(got, ref), TRACE_TOL) < TRACE_TOL
    first = lines(cache)
    assert len(first) == 1, first
    key, choice = first[0].split(":")
    S, TZ, G, PF, PR, SR, TZR, RS, FS = (int(t) for t in choice.split())
    q = B.fwi_exec_query(w.grid, w.geom, ex, B.WS_FORWARD)
    assert q["shots_in_flight"] == min(S, w.geom.nshot)
    assert chosen(q) == (TZ, G, PF, PR)

    # a different, valid choice under the same key; the library must take it
    # from the file once it has forgotten its own
    TZ2 = 32 if TZ != 32 else 16
    PF2 = 7 if PF != 7 else 3
    with open(cache, "w") as f:
        f.write(f"{key}: {S} {TZ2} {G} {PF2} 3 {SR} {TZR} {RS} {FS}\n")
    B.fwi_tune_reset()
    assert chosen(B.fwi_exec_query(w.grid, w.geom, ex, B.WS_FORWARD)) == (TZ2, G, PF2, 3)
    got2 = B.forward(w.v_true, w.wavelet, w.grid, w.geom, ex).cpu().numpy()
    assert len(lines(cache)) == 1, "tuned again instead of reading the file"
    assert report("forward tiny autotuned (from file)", rel(got2, ref), TRACE_TOL) < TRACE_TOL

    # an unreadable line is ignored: the call tunes again and appends a line
    with open(cache, "w") as f:
        f.write(f"{key}: 0 0 0 5 9 0 0 7\n")
    B.fwi_tune_reset()
    got3 = B.forward(w.v_true, w.wavelet, w.grid, w.geom, ex).cpu().numpy()
    assert len(lines(cache)) == 2
    assert report("forward tiny autotuned (bad line)", rel(got3, ref), TRACE_TOL) < TRACE_TOL
