"""GPU parity at full grid sizes against stored FP64 oracle values.

The oracle values come from tests/golden/make_golden.py (oracle only) and
hold a regular subsample of the outputs; the GPU runs the same inputs,
regenerated here from the same seeds, in the batched launch configurations
the benchmark uses, and the subsample is compared with the same relative-L2
tolerances as the small cases.
"""
import os
import sys

import numpy as np
import pytest

from paper_1406_1864_amd import binding as B

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_golden  # noqa: E402

from helpers import GRAD_TOL, TRACE_TOL, rel, report

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def golden(name):
    path = os.path.join(HERE, "golden", name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"stored oracle values {name}.npz not generated (tests/golden/make_golden.py {name})")
    z = np.load(path)
    w, grid, geom, wav, seed = make_golden.case_inputs(name)
    from paper_1406_1864_amd.synthetic import random_traces
    d_obs = random_traces(geom, grid.nt_max, seed=seed, scale=float(z["scale"]))
    return z, w, grid, geom, wav, d_obs


def check(tag, z, J, g, H1, traces, mult=1.0, D=None):
    """The stored residual is well conditioned (recorded data = 0.3 x RMS
    noise), so J is held to the seismogram tolerance."""
    zs, rs, ts = int(z["zs"]), int(z["rs"]), int(z["ts"])
    ntr = z["traces"].shape[0]
    assert report(f"{tag} traces", rel(traces[::rs, ::ts][:ntr], z["traces"]), TRACE_TOL) < TRACE_TOL
    assert report(f"{tag} J", abs(J - mult * float(z["J"])) / (mult * float(z["J"])), TRACE_TOL) <= TRACE_TOL
    assert report(f"{tag} grad", rel(g[::zs, ::zs], mult * z["g"]), GRAD_TOL) < GRAD_TOL
    assert report(f"{tag} H1", rel(H1[::zs, ::zs], mult * z["H1"]), GRAD_TOL) < GRAD_TOL
    if D is not None:
        assert report(f"{tag} D", rel(D[::4, ::zs, ::zs], mult * z["D"]), GRAD_TOL) < GRAD_TOL


@pytest.mark.parametrize("S,TZ", [(8, 64), (8, 32), (8, 128), (4, 64)])
def test_layered_1024x384_short_record(S, TZ):
    """8 shots = the 2 stored shots repeated 4 times, so that the batched
    launch fills 8 slots (one per XCD) and the result is 4x the oracle's."""
    name = "layered_1024x384_nt400"
    z, w, grid, geom2, wav, d2 = golden(name)
    geom = geom2.subset([0, 1] * 4)
    d_obs = np.concatenate([d2] * 4)
    ex = B.make_exec(shots_in_flight=S, tile_rows=TZ)
    tr = B.forward(w.v_start, wav, grid, geom, ex).cpu().numpy()
    J, g, H1, _ = B.gradient(w.v_start, wav, grid, geom, d_obs, "int", ex)
    rs = int(z["rs"])
    nrec = geom2.rec_ptr[1]
    both = np.concatenate([tr[0:nrec:rs], tr[nrec:2 * nrec:rs]])
    check(f"layered nt400 S{S} TZ{TZ}", z, float(J), g.cpu().numpy(), H1.cpu().numpy(),
          np.repeat(both, rs, axis=0), mult=4.0)


@pytest.mark.parametrize("mode", ["batched", "plain", "two_step", "two_step_pf3", "fwd_two_step"])
def test_layered_1024x384_full_record(mode):
    z, w, grid, geom, wav, d_obs = golden("layered_1024x384_nt4000")
    ex = {"plain": B.make_exec(mode=B.EXEC_PLAIN), "batched": B.make_exec(autotune=1),
          "two_step": B.make_exec(reverse_steps=2, tile_rows_reverse=16),
          "two_step_pf3": B.make_exec(reverse_steps=2, tile_rows_reverse=32, prefetch_reverse=3),
          "fwd_two_step": B.make_exec(forward_steps=2, reverse_steps=2, tile_rows=32, tile_rows_reverse=32)}[mode]
    tr = B.forward(w.v_start, wav, grid, geom, ex).cpu().numpy()
    J, g, H1, _ = B.gradient(w.v_start, wav, grid, geom, d_obs, "int", ex)
    check(f"layered nt4000 {mode}", z, float(J), g.cpu().numpy(), H1.cpu().numpy(), tr)


def test_layered_2048x768_full_record_offset_diag():
    z, w, grid, geom, wav, d_obs = golden("layered_2048x768_nt8000")
    ex = B.make_exec(autotune=1)
    tr = B.forward(w.v_start, wav, grid, geom, ex).cpu().numpy()
    J, g, H1, D = B.gradient(w.v_start, wav, grid, geom, d_obs, "int", ex, hmax=int(z["hmax"]))
    check("layered 2048x768 nt8000", z, float(J), g.cpu().numpy(), H1.cpu().numpy(), tr, D=D.cpu().numpy())


@pytest.mark.parametrize("steps", [0, 2, 22])
def test_ragged_1024x384_extremes_batched(steps):
    """The shortest (nt 2013, 264 receivers) and the longest (nt 5988, 798
    receivers) record of the 256-shot ragged workload, each repeated 4 times:
    one batch of 8 uneven shots (sorted by record length, idle launches for the
    short ones) in the autotuned batched launch (and with two reverse steps per
    launch, where the two record lengths differ in parity); 4x the oracle's
    values."""
    z, w, grid, geom2, wav, d2 = golden("ragged_1024x384_extremes")
    geom = geom2.subset([0, 1] * 4)
    d_obs = np.concatenate([d2] * 4)
    # 22: two forward and two reverse steps per launch
    ex = B.make_exec(autotune=1, reverse_steps=steps % 10, forward_steps=steps // 10)
    tr = B.forward(w.v_start, wav, grid, geom, ex).cpu().numpy()
    J, g, H1, _ = B.gradient(w.v_start, wav, grid, geom, d_obs, "int", ex)
    check("ragged extremes x4", z, float(J), g.cpu().numpy(), H1.cpu().numpy(), tr[:geom2.ntrace], mult=4.0)
    assert np.all(tr[:geom2.rec_ptr[1], int(geom2.nt[0]):] == 0)


@pytest.mark.parametrize("steps", [1, 2])
def test_layered_1024x384_extended_image(steps):
    """Offset-extended image |h| <= 16 at full grid size: 8 shots (the 2
    stored ones repeated 4 times) in one batch of 8 slots with graph chunks,
    so the result is 4x the oracle's; every 4th offset slice is compared.
    With one or two time steps per forward and reverse launch."""
    name = "layered_1024x384_nt400_ext16"
    z, w, grid, geom2, wav, d2 = golden(name)
    geom = geom2.subset([0, 1] * 4)
    d_obs = np.concatenate([d2] * 4)
    hmax, hs, zs = int(z["hmax"]), int(z["hs"]), int(z["zs"])
    ex = B.make_exec(shots_in_flight=8, tile_rows=16, graph_steps=32, reverse_steps=steps, forward_steps=steps)
    J, g, image = B.extended_image(w.v_start, wav, grid, geom, d_obs, hmax, "int", ex)
    assert report("layered nt400 ext J", abs(float(J) - 4 * float(z["J"])) / (4 * float(z["J"])), TRACE_TOL) \
        <= TRACE_TOL
    sub = image.cpu().numpy()[::hs, ::zs, ::zs]
    for k in range(sub.shape[0]):
        h = k * hs - hmax
        assert report(f"layered nt400 ext image h={h}", rel(sub[k], 4 * z["I"][k]), GRAD_TOL) < GRAD_TOL, h
