"""The autograd pair J(v) at full size: the 1024x384 layered model with 32
shots and nt 4000 (the differentiation workload: shots 0, 2, ..., 62 of the
layered benchmark), run with the launch settings the benchmark's autotuner
picks (two-step launches, large reverse groups, every shot's checkpoints
kept between forward and backward).

* Oracle parity: the stored FP64 oracle values of one layered shot
  (tests/golden/layered_1024x384_nt4000.npz, recorded data = seeded noise)
  replicated 32 times, so that J, the gradient and H1 are 32 times the
  oracle's; compared on the stored subsample of cells, receivers and samples.
* Directional derivatives of the GPU's own J: central differences at
  eps = 1e-3 relative along a Gaussian bump (sigma 16 cells, mid-depth) and
  along seeded smoothed noise (sigma 8 cells, tapered to zero within 12 cells
  of the edges), against <dJ/dv, dv>, within 1e-2 (FP32 traces limit the
  accuracy of the difference quotient).
"""
import os
import sys

import numpy as np
import pytest

from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import autograd_1024x384, bump_direction, noise_direction

from helpers import GRAD_TOL, J_TOL, TRACE_TOL, rel, report

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1406_1864_amd.autograd import FWIProblem, fwi_misfit  # noqa: E402
from test_gpu_fullsize import golden  # noqa: E402

REPEAT = 32


def test_autograd_1024x384_32_shots_against_oracle():
    z, w, grid, geom1, wav, d1 = golden("layered_1024x384_nt4000")
    geom = geom1.subset([0] * REPEAT)
    d_obs = np.concatenate([d1] * REPEAT)
    ex = B.make_exec(autotune=1)
    pr = FWIProblem(grid, geom, wav, d_obs, "int", ex, illum=True)
    v = torch.tensor(w.v_start, device="cuda", requires_grad=True)
    J = fwi_misfit(v, pr)
    J.backward()
    chosen = B.fwi_exec_query(grid, pr.geom, ex, B.WS_AUTOGRAD)
    print(f"[autograd 1024x384 x{REPEAT}] launch settings {chosen}", flush=True)
    zs, rs, ts = int(z["zs"]), int(z["rs"]), int(z["ts"])
    tag = f"autograd 1024x384 nt4000 x{REPEAT}"
    Jref = REPEAT * float(z["J"])
    assert report(f"{tag} J", abs(float(J) - Jref) / Jref, J_TOL) <= J_TOL
    g = v.grad.cpu().numpy()
    H1 = pr.illum.cpu().numpy()
    assert report(f"{tag} grad", rel(g[::zs, ::zs], REPEAT * z["g"]), GRAD_TOL) < GRAD_TOL
    assert report(f"{tag} H1", rel(H1[::zs, ::zs], REPEAT * z["H1"]), GRAD_TOL) < GRAD_TOL
    # traces of the same engine and settings (the forward sweep of J)
    tr = B.forward(w.v_start, wav, grid, geom1, ex).cpu().numpy()
    ntr = z["traces"].shape[0]
    assert report(f"{tag} traces", rel(tr[::rs, ::ts][:ntr], z["traces"]), TRACE_TOL) < TRACE_TOL


@pytest.fixture(scope="module")
def c4():
    w = autograd_1024x384()
    d_obs = B.forward(w.v_true, w.wavelet, w.grid, w.geom, B.make_exec())
    pr = FWIProblem(w.grid, w.geom, w.wavelet, d_obs, "int", B.make_exec(autotune=1), illum=False)
    v = torch.tensor(w.v_start, device="cuda", requires_grad=True)
    J = fwi_misfit(v, pr)
    J.backward()
    return w, pr, v.grad.detach().double()


@pytest.mark.parametrize("direction", ["bump", "noise"])
def test_autograd_1024x384_directional_fd(c4, direction):
    w, pr, grad = c4
    nz, nx = w.grid.nz, w.grid.nx
    d = bump_direction(nz, nx, sigma=16.0) if direction == "bump" else noise_direction(nz, nx, seed=2014)
    eps = 1e-3
    v0 = w.v_start.astype(np.float64)
    vp = torch.tensor(v0 * (1 + eps * d / np.abs(d).max()), dtype=torch.float32, device="cuda")
    vm = torch.tensor(v0 * (1 - eps * d / np.abs(d).max()), dtype=torch.float32, device="cuda")
    dv = (vp.double() - vm.double()) / 2.0       # the float32 perturbation actually applied
    lin = float((grad * dv).sum())
    with torch.no_grad():
        fd = (float(fwi_misfit(vp, pr)) - float(fwi_misfit(vm, pr))) / 2.0
    assert report(f"autograd 1024x384 FD {direction}", abs(fd - lin) / abs(lin), 1e-2) <= 1e-2, (fd, lin)
