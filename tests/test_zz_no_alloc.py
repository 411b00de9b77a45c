"""fwi_gradient_static, the gradient entry point that allocates nothing (its
scratch is a static device array per GPU), against fwi_gradient with a
caller-owned workspace: two calls in a row, the second on a smaller problem,
each to the hot path's tolerances (J 1e-4, gradient and Hessian diagonals
1e-3 relative L2)."""
import numpy as np
import pytest

from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import random_traces, tiny_24x16

from helpers import GRAD_TOL, J_TOL, rel, report
from test_gpu_parity import ragged_geometry

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def cases():
    grid, geom, v_true, v_start, wav = ragged_geometry()                 # 64x48, 5 uneven shots
    big = (grid, geom, v_start, wav, random_traces(geom, grid.nt_max, seed=41, scale=1e-3), 2)
    w = tiny_24x16(nt=200)                                                # 24x16, 2 shots, nt 200
    small = (w.grid, w.geom, w.v_start, w.wavelet, random_traces(w.geom, w.grid.nt_max, seed=42, scale=1e-3), 1)
    return [("ragged 64x48", big), ("tiny 24x16", small)]


def static_gradient(grid, geom, v, wav, d_obs, hmax, misfit="int"):
    vd = torch.as_tensor(np.asarray(v, np.float32), device="cuda")
    w, wst = B._wavelet(wav, grid.nt_max, "cuda")
    dobs = torch.as_tensor(np.asarray(d_obs, np.float32), device="cuda")
    J = torch.empty((), dtype=torch.float64, device="cuda")
    g = torch.empty((grid.nz, grid.nx), dtype=torch.float32, device="cuda")
    H1 = torch.empty_like(g)
    D = torch.empty((2 * hmax + 1, grid.nz, grid.nx), dtype=torch.float32, device="cuda")
    B.fwi_gradient_static(grid, geom, None, vd, w, wst, dobs, misfit, J, g, H1, hmax, "pm", D)
    return J, g, H1, D


def test_static_gradient_matches_workspace_gradient_on_two_calls():
    for tag, (grid, geom, v, wav, d_obs, hmax) in cases():
        need = B.fwi_workspace_bytes(grid, geom, B.make_exec(graph_steps=-1), B.WS_GRADIENT, hmax)
        assert 0 < need <= B.FWI_STATIC_SCRATCH_BYTES, (tag, need)
        Js, gs, Hs, Ds = static_gradient(grid, geom, v, wav, d_obs, hmax)
        Jr, gr, Hr, Dr = B.gradient(v, wav, grid, geom, d_obs, "int", hmax=hmax)
        torch.cuda.synchronize()
        Jr = float(Jr)
        assert report(f"static J {tag}", abs(float(Js) - Jr) / Jr, J_TOL) <= J_TOL
        assert report(f"static grad {tag}", rel(gs.cpu().numpy(), gr.cpu().numpy()), GRAD_TOL) < GRAD_TOL
        assert report(f"static H1 {tag}", rel(Hs.cpu().numpy(), Hr.cpu().numpy()), GRAD_TOL) < GRAD_TOL
        assert report(f"static D {tag}", rel(Ds.cpu().numpy(), Dr.cpu().numpy()), GRAD_TOL) < GRAD_TOL
