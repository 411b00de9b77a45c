"""GPU parity of the offset-extended image (fwi_extended_image) against the
FP64 oracle: every offset slice to the gradient tolerance (relative L2
1e-3), J to the tolerance its seismograms imply, and the h = 0 slice against
the gradient of the same call."""
import numpy as np
import pytest

import oracle
from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import anomaly_200x100, random_traces, tiny_24x16

from helpers import GRAD_TOL, j_tolerance, rel, report
from test_gpu_parity import EXECS, cpu, ragged_geometry

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def check(tag, ref, got, J_ref, jt, hmax):
    J, g, image = got
    image = cpu(image)
    assert image.shape == ref.shape
    assert report(f"ext J {tag}", abs(float(J) - J_ref) / J_ref, jt) <= jt
    for h in range(2 * hmax + 1):
        assert report(f"ext image {tag} h={h - hmax}", rel(image[h], ref[h]), GRAD_TOL) < GRAD_TOL, h
    # h = 0 is the gradient: same products, summed in another order
    assert report(f"ext image {tag} h=0 vs grad", rel(image[hmax], cpu(g)), 1e-5) < 1e-5
    for h in range(1, hmax + 1):
        assert np.all(image[hmax + h][:, :h] == 0) and np.all(image[hmax - h][:, -h:] == 0)


@pytest.mark.parametrize("name", list(EXECS))
@pytest.mark.parametrize("kind", ["int", "l2"])
def test_extended_image_tiny(name, kind):
    w = tiny_24x16(nt=300)
    hmax = 4
    d_obs = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    J, ref = oracle.extended_image(w.v_start, w.grid, w.geom, w.wavelet, d_obs, kind, hmax)
    got = B.extended_image(w.v_start, w.wavelet, w.grid, w.geom, d_obs.astype(np.float32), hmax, kind, EXECS[name])
    syn = oracle.forward_traces(w.v_start, w.grid, w.geom, w.wavelet)
    check(f"tiny {kind} {name}", ref, got, J, j_tolerance(syn, d_obs, kind, w.grid.dt), hmax)


@pytest.mark.parametrize("name", list(EXECS))
def test_extended_image_ragged(name):
    """Uneven record lengths (one shot of 2 samples), a shot without
    receivers, several windows of reverse steps per batch."""
    grid, geom, v_true, v_start, wav = ragged_geometry()
    hmax = 8
    d_obs = oracle.forward_traces(v_true, grid, geom, wav)
    J, ref = oracle.extended_image(v_start, grid, geom, wav, d_obs, "int", hmax)
    got = B.extended_image(v_start, wav, grid, geom, d_obs.astype(np.float32), hmax, "int", EXECS[name])
    syn = oracle.forward_traces(v_start, grid, geom, wav)
    check(f"ragged {name}", ref, got, J, j_tolerance(syn, d_obs, "int", grid.dt), hmax)


def test_extended_image_anomaly_full():
    """The 200x100 anomaly workload (nt 1000), offsets up to 16 cells."""
    w = anomaly_200x100()
    hmax = 16
    d_obs = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    J, ref = oracle.extended_image(w.v_start, w.grid, w.geom, w.wavelet, d_obs, "int", hmax)
    got = B.extended_image(w.v_start, w.wavelet, w.grid, w.geom, d_obs.astype(np.float32), hmax, "int")
    syn = oracle.forward_traces(w.v_start, w.grid, w.geom, w.wavelet)
    check("anomaly 200x100", ref, got, J, j_tolerance(syn, d_obs, "int", w.grid.dt), hmax)


def test_extended_image_repeated_calls_agree():
    """The offset sums start from zero on every call (same workspace)."""
    grid, geom, v_true, v_start, wav = ragged_geometry()
    d_obs = random_traces(geom, grid.nt_max, seed=3, scale=1e-3)
    ex = EXECS["batched_graph"]
    ws = B.workspace(grid, geom, B.WS_EXTIMAGE, ex, 6)
    a = B.extended_image(v_start, wav, grid, geom, d_obs, 6, "int", ex, ws=ws)
    b = B.extended_image(v_start, wav, grid, geom, d_obs, 6, "int", ex, ws=ws)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
