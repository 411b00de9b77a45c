"""torch.autograd.Function J(v): forward/backward through the HIP library,
checked against the FP64 oracle and against directional finite differences."""
import numpy as np
import pytest

import oracle
from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import anomaly_200x100, bump_direction, tiny_24x16

from helpers import GRAD_TOL, j_tolerance, rel, report

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1406_1864_amd.autograd import FWIProblem, fwi_misfit  # noqa: E402


@pytest.fixture(scope="module")
def anomaly():
    w = anomaly_200x100()
    d_obs = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    J, g, H1, E = oracle.gradient(w.v_start, w.grid, w.geom, w.wavelet, d_obs, "int", return_parts=True)
    syn = oracle.forward_traces(w.v_start, w.grid, w.geom, w.wavelet)
    return w, d_obs, (J, g, H1, E, syn)


@pytest.mark.parametrize("exec_", [None, B.make_exec(graph_steps=-1), B.make_exec(mode=B.EXEC_PLAIN),
                                   B.make_exec(shots_in_flight=2, shots_in_flight_reverse=1, tile_rows_reverse=12),
                                   B.make_exec(reverse_steps=2, graph_steps=7),
                                   B.make_exec(forward_steps=2, reverse_steps=2, graph_steps=6)])
def test_autograd_matches_oracle(anomaly, exec_):
    w, d_obs, (J, g, H1, E, syn) = anomaly
    pr = FWIProblem(w.grid, w.geom, w.wavelet, d_obs.astype(np.float32), "int", exec_, hmax=4)
    v = torch.tensor(w.v_start, device="cuda", requires_grad=True)
    Jg = fwi_misfit(v, pr)
    assert Jg.dtype == torch.float64
    jt = j_tolerance(syn, d_obs, "int", w.grid.dt)
    assert report("autograd J", abs(float(Jg) - J) / J, jt) <= jt
    (3.0 * Jg).backward()
    assert report("autograd grad", rel(v.grad.cpu().numpy(), 3.0 * g), GRAD_TOL) < GRAD_TOL
    assert report("autograd H1", rel(pr.illum.cpu().numpy(), H1), GRAD_TOL) < GRAD_TOL
    A = [oracle.aperture_factor(w.grid, *w.geom.shot(0)[2:4])]
    Dref = oracle.offset_diag(w.v_start, E, A, 4)
    assert report("autograd D", rel(pr.offset.cpu().numpy(), Dref), GRAD_TOL) < GRAD_TOL


@pytest.mark.parametrize("exec_", [
    B.make_exec(shots_in_flight=1, shots_in_flight_reverse=3, reverse_steps=2, graph_steps=5),
    B.make_exec(shots_in_flight=2, shots_in_flight_reverse=4, tile_rows_reverse=8, graph_steps=-1),
    # two forward steps per launch as well (odd and even record lengths)
    B.make_exec(shots_in_flight=2, shots_in_flight_reverse=5, reverse_steps=2, forward_steps=2, graph_steps=3)])
def test_autograd_ragged_reverse_groups(exec_):
    """The autograd pair keeps every shot's checkpoints, so its reverse sweep
    groups the shots on its own: groups larger than the forward batches, the
    last one partly idle, uneven record lengths (5 shots)."""
    from test_gpu_parity import ragged_geometry
    grid, geom, v_true, v_start, wav = ragged_geometry()
    d_obs = oracle.forward_traces(v_true, grid, geom, wav)
    J, g, H1 = oracle.gradient(v_start, grid, geom, wav, d_obs, "int")
    pr = FWIProblem(grid, geom, wav, d_obs.astype(np.float32), "int", exec_)
    v = torch.tensor(v_start, device="cuda", requires_grad=True)
    Jg = fwi_misfit(v, pr)
    Jg.backward()
    syn = oracle.forward_traces(v_start, grid, geom, wav)
    jt = j_tolerance(syn, d_obs, "int", grid.dt)
    assert report("autograd ragged groups J", abs(float(Jg) - J) / J, jt) <= jt
    assert report("autograd ragged groups grad", rel(v.grad.cpu().numpy(), g), GRAD_TOL) < GRAD_TOL
    assert report("autograd ragged groups H1", rel(pr.illum.cpu().numpy(), H1), GRAD_TOL) < GRAD_TOL


def test_autograd_equals_fused_gradient(anomaly):
    """The split forward/backward and the fused fwi_gradient give the same
    numbers (same kernels, same order)."""
    w, d_obs, _ = anomaly
    ex = B.make_exec(shots_in_flight=1)
    pr = FWIProblem(w.grid, w.geom, w.wavelet, d_obs.astype(np.float32), "l2", ex)
    v = torch.tensor(w.v_start, device="cuda", requires_grad=True)
    J = fwi_misfit(v, pr)
    J.backward()
    J2, g2, H2, _ = B.gradient(w.v_start, w.wavelet, w.grid, w.geom, d_obs.astype(np.float32), "l2", ex)
    assert float(J) == float(J2)
    assert torch.equal(v.grad, g2)
    assert torch.equal(pr.illum, H2)


def test_directional_derivative_gpu_fd(anomaly):
    """<dJ/dv, d> against central differences of the GPU's own J
    (eps = 1e-3 relative; FP32 traces limit the FD accuracy to ~1e-3)."""
    w, d_obs, _ = anomaly
    pr = FWIProblem(w.grid, w.geom, w.wavelet, d_obs.astype(np.float32), "int")
    d = bump_direction(w.grid.nz, w.grid.nx, sigma=16.0)
    d[:12, :] = d[-12:, :] = 0.0
    d[:, :12] = d[:, -12:] = 0.0
    v0 = torch.tensor(w.v_start, device="cuda", requires_grad=True)
    J = fwi_misfit(v0, pr)
    J.backward()
    lin = float((v0.grad.double() * torch.as_tensor(d, device="cuda")).sum())
    eps = 1e-3
    vp = torch.tensor(w.v_start * (1 + eps * d / np.abs(d).max()), dtype=torch.float32, device="cuda")
    vm = torch.tensor(w.v_start * (1 - eps * d / np.abs(d).max()), dtype=torch.float32, device="cuda")
    dv = (vp.double() - vm.double()).cpu().numpy() / 2.0   # exact float32 perturbation actually applied
    lin_exact = float((v0.grad.double().cpu().numpy() * dv).sum())
    Jp = float(fwi_misfit(vp, pr))
    Jm = float(fwi_misfit(vm, pr))
    fd = (Jp - Jm) / 2.0
    assert report("gpu FD directional", abs(fd - lin_exact) / abs(lin_exact), 1e-2) <= 1e-2, (fd, lin_exact, lin)


def test_directional_derivative_against_oracle_fd():
    """<dJ/dv, d> of the GPU against the FP64 oracle's central difference."""
    w = tiny_24x16(nt=300)
    d_obs = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    rng = np.random.default_rng(21)
    d = rng.standard_normal((w.grid.nz, w.grid.nx))
    d[0, :] = d[-1, :] = 0.0
    d[:, 0] = d[:, -1] = 0.0
    v0 = w.v_start.astype(np.float64)
    eps = 1e-4

    def Jo(v):
        return oracle.misfit(oracle.forward_traces(v, w.grid, w.geom, w.wavelet), d_obs, "int", w.grid.dt)[0]

    fd = (Jo(v0 + eps * d * v0) - Jo(v0 - eps * d * v0)) / (2 * eps)
    pr = FWIProblem(w.grid, w.geom, w.wavelet, d_obs.astype(np.float32), "int")
    v = torch.tensor(w.v_start, device="cuda", requires_grad=True)
    fwi_misfit(v, pr).backward()
    lin = float(np.sum(v.grad.cpu().numpy().astype(np.float64) * d * v0))
    assert report("oracle FD directional", abs(lin - fd) / abs(fd), 1e-3) <= 1e-3


def test_backward_requires_matching_forward(anomaly):
    w, d_obs, _ = anomaly
    pr = FWIProblem(w.grid, w.geom, w.wavelet, d_obs.astype(np.float32), "int")
    v = torch.tensor(w.v_start, device="cuda")
    grad = torch.empty_like(v)
    other = torch.tensor(w.v_start, device="cuda")
    J = torch.empty((), dtype=torch.float64, device="cuda")
    B.fwi_misfit_forward(w.grid, pr.geom, None, v, pr.wavelet, 0, pr.d_obs, "int", J, pr.ws, pr.ws.numel())
    with pytest.raises(B.FwiError) as e:
        B.fwi_misfit_backward(w.grid, pr.geom, None, other, pr.wavelet, 0, None, grad, None, 0, "pm", None,
                              pr.ws, pr.ws.numel())
    assert e.value.code == B.FWI_ERR_STATE
