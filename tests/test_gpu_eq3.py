"""Eq. (3) taken literally on the GPU (fwi_gradient with
FWI_MISFIT_EQ3_LITERAL) against the FP64 oracle, and the end-of-record term
that separates it from the exact eq. (2) gradient, measured as the difference
of the two GPU gradients."""
import numpy as np
import pytest

import oracle
from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import anomaly_200x100, tiny_24x16

from helpers import GRAD_TOL, j_tolerance, rel, report
from test_gpu_parity import EXECS, cpu, ragged_geometry

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def run(tag, v, grid, geom, wav, d_obs, ex=None):
    J3, g3 = oracle.gradient_eq3_literal(v, grid, geom, wav, d_obs)
    Jg, gg, _, _ = B.gradient(v, wav, grid, geom, d_obs.astype(np.float32), "eq3", ex, illum=False)
    syn = oracle.forward_traces(v, grid, geom, wav)
    jt = j_tolerance(syn, d_obs, "int", grid.dt)
    assert report(f"eq3 J {tag}", abs(float(Jg) - J3) / J3, jt) <= jt
    assert report(f"eq3 grad {tag}", rel(cpu(gg), g3), GRAD_TOL) < GRAD_TOL
    return cpu(gg)


@pytest.mark.parametrize("name", list(EXECS))
def test_eq3_literal_tiny(name):
    w = tiny_24x16(nt=300)
    d_obs = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    run(f"tiny {name}", w.v_start, w.grid, w.geom, w.wavelet, d_obs, EXECS[name])


@pytest.mark.parametrize("name", list(EXECS))
def test_eq3_literal_ragged(name):
    grid, geom, v_true, v_start, wav = ragged_geometry()
    d_obs = oracle.forward_traces(v_true, grid, geom, wav)
    run(f"ragged {name}", v_start, grid, geom, wav, d_obs, EXECS[name])


def test_eq3_end_of_record_term_anomaly_full():
    """200x100 anomaly, nt 1000: g_int - g3 from the GPU equals the oracle's
    end-of-record term; its size relative to the gradient is reported."""
    w = anomaly_200x100()
    d_obs = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    g3 = run("anomaly 200x100", w.v_start, w.grid, w.geom, w.wavelet, d_obs)
    _, g, _, _ = B.gradient(w.v_start, w.wavelet, w.grid, w.geom, d_obs.astype(np.float32), "int", illum=False)
    g = cpu(g).astype(np.float64)
    E = oracle.end_of_record_term(w.v_start, w.grid, w.geom, w.wavelet, d_obs)
    share = np.linalg.norm(E) / np.linalg.norm(g)
    print(f"[eq3] end-of-record term / exact gradient (rel. L2): {share:.3e}")
    tol = GRAD_TOL * max(1.0, 1.0 / share)
    assert report("eq3 end-of-record term", rel(g - g3, E), tol) < tol
