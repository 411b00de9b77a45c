"""GPU parity with the free-surface option (odd image above the model, no
top sponge) against the FP64 oracle: forward traces (1e-4), gradients and
Hessian diagonals (1e-3), through the batched, graph and plain launches, the
autograd pair, Born modelling and the Gauss-Newton product."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import anomaly_200x100, tiny_24x16

from helpers import GRAD_TOL, TRACE_TOL, j_tolerance, rel, report
from test_gpu_parity import EXECS, cpu, ragged_geometry

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def fs(grid):
    return dataclasses.replace(grid, free_surface=True)


@pytest.mark.parametrize("name", list(EXECS))
def test_free_surface_forward_tiny(name):
    w = tiny_24x16(nt=300)
    grid = fs(w.grid)
    ref = oracle.forward_traces(w.v_true, grid, w.geom, w.wavelet)
    got = cpu(B.forward(w.v_true, w.wavelet, grid, w.geom, EXECS[name]))
    assert report(f"fs forward tiny {name}", rel(got, ref), TRACE_TOL) < TRACE_TOL
    absorbing = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    assert rel(got, absorbing) > 0.05        # the surface reflection is there


@pytest.mark.parametrize("name", list(EXECS))
@pytest.mark.parametrize("kind", ["int", "l2"])
def test_free_surface_gradient_ragged(name, kind):
    """Receivers on the top row, a source in the top corner cell."""
    grid, geom, v_true, v_start, wav = ragged_geometry()
    grid = fs(grid)
    d_obs = oracle.forward_traces(v_true, grid, geom, wav)
    J, g, H1 = oracle.gradient(v_start, grid, geom, wav, d_obs, kind)
    Jg, gg, Hg, _ = B.gradient(v_start, wav, grid, geom, d_obs.astype(np.float32), kind, EXECS[name])
    syn = oracle.forward_traces(v_start, grid, geom, wav)
    jt = j_tolerance(syn, d_obs, kind, grid.dt)
    tag = f"fs ragged {kind} {name}"
    assert report(f"J {tag}", abs(float(Jg) - J) / J, jt) <= jt
    assert report(f"grad {tag}", rel(cpu(gg), g), GRAD_TOL) < GRAD_TOL
    assert report(f"H1 {tag}", rel(cpu(Hg), H1), GRAD_TOL) < GRAD_TOL


def test_free_surface_anomaly_full_autograd():
    """200x100 anomaly, nt 1000, through the autograd pair."""
    from paper_1406_1864_amd.autograd import FWIProblem, fwi_misfit
    w = anomaly_200x100()
    grid = fs(w.grid)
    d_obs = oracle.forward_traces(w.v_true, grid, w.geom, w.wavelet)
    J, g, H1 = oracle.gradient(w.v_start, grid, w.geom, w.wavelet, d_obs, "int")
    pr = FWIProblem(grid, w.geom, w.wavelet, d_obs.astype(np.float32), "int", None)
    v = torch.tensor(w.v_start, device="cuda", requires_grad=True)
    Jg = fwi_misfit(v, pr)
    Jg.backward()
    syn = oracle.forward_traces(w.v_start, grid, w.geom, w.wavelet)
    jt = j_tolerance(syn, d_obs, "int", grid.dt)
    assert report("fs anomaly autograd J", abs(float(Jg) - J) / J, jt) <= jt
    assert report("fs anomaly autograd grad", rel(v.grad.cpu().numpy(), g), GRAD_TOL) < GRAD_TOL
    assert report("fs anomaly autograd H1", rel(pr.illum.cpu().numpy(), H1), GRAD_TOL) < GRAD_TOL


def test_free_surface_born_and_gn_hvp_tiny():
    w = tiny_24x16(nt=300)
    grid = fs(w.grid)
    rng = np.random.default_rng(21)
    dv = rng.standard_normal((grid.nz, grid.nx)) * 20.0
    ref = oracle.born(w.v_start, grid, w.geom, w.wavelet, dv)
    got = cpu(B.born(w.v_start, w.wavelet, grid, w.geom, dv, EXECS["batched_graph"]))
    assert report("fs born tiny", rel(got, ref), TRACE_TOL) < TRACE_TOL
    Jb, H = oracle.gn_hvp(w.v_start, grid, w.geom, w.wavelet, dv, "int")
    Jg, Hg = B.gn_hvp(w.v_start, w.wavelet, grid, w.geom, dv, "int", EXECS["batched_graph"])
    assert report("fs gn J tiny", abs(float(Jg) - Jb) / Jb, TRACE_TOL) <= TRACE_TOL
    assert report("fs gn H dv tiny", rel(cpu(Hg), H), GRAD_TOL) < GRAD_TOL
