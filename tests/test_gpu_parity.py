"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative L2): 1e-4 on seismograms, 1e-3 on gradients and
Hessian diagonals; J to the tolerance its seismograms imply (tests/helpers.py).
"""
import numpy as np
import pytest

import oracle
from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import (Geometry, Grid, anomaly_200x100, gaussian_anomaly, ricker,
                                           tiny_24x16, random_traces)

from helpers import GRAD_TOL, TRACE_TOL, j_tolerance, rel, report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def cpu(t):
    return t.detach().cpu().numpy()


EXECS = {
    "plain": B.make_exec(mode=B.EXEC_PLAIN),
    "batched_direct": B.make_exec(shots_in_flight=2, graph_steps=-1, tile_rows=16),
    "batched_graph": B.make_exec(shots_in_flight=3, graph_steps=7, tile_rows=24),
    # the reverse sweep takes each forward batch two shots at a time, 8-row tiles
    "split_config": B.make_exec(shots_in_flight=4, shots_in_flight_reverse=2, tile_rows=16, tile_rows_reverse=8,
                                graph_steps=5),
    # two reverse steps per launch, direct launches and graph chunks (the
    # latter with loads three rows ahead)
    "two_step": B.make_exec(shots_in_flight=3, tile_rows=16, graph_steps=-1, reverse_steps=2),
    "two_step_graph": B.make_exec(shots_in_flight=4, shots_in_flight_reverse=2, tile_rows=24, tile_rows_reverse=12,
                                  graph_steps=5, reverse_steps=2, prefetch_reverse=3),
    # two forward steps per launch (with one-step and two-step reverse sweeps)
    "fwd_two_step": B.make_exec(shots_in_flight=3, tile_rows=16, graph_steps=-1, forward_steps=2),
    "both_two_step_graph": B.make_exec(shots_in_flight=4, shots_in_flight_reverse=2, tile_rows=12,
                                       tile_rows_reverse=24, graph_steps=5, reverse_steps=2, forward_steps=2,
                                       prefetch=3),
    # graph chunks of the two-step sweeps as one launch chain, and as three
    # chains over uneven shares of the shots (1, 2, 2 of the ragged case's 5)
    "two_step_one_chain": B.make_exec(shots_in_flight=4, tile_rows=16, tile_rows_reverse=16, graph_steps=5,
                                      reverse_steps=2, forward_steps=2, graph_branches=1),
    "two_step_three_chains": B.make_exec(shots_in_flight=5, tile_rows=16, tile_rows_reverse=8, graph_steps=3,
                                         reverse_steps=2, forward_steps=2, graph_branches=3),
}


def ragged_geometry():
    """64x48 model, 5 shots: uneven record lengths and apertures, a shot with
    no receivers, receivers on a line, in a vertical well and at the model
    corners and edges; the source of one shot sits on a corner cell."""
    nz, nx = 48, 64
    rec_iz, rec_ix, ptr = [], [], [0]
    spreads = [
        [(2, x) for x in range(0, 64, 3)],                    # surface line
        [(z, 40) for z in range(0, 48, 2)] + [(47, 63), (0, 0)],  # well + corners
        [],                                                   # no receivers
        [(5, x) for x in range(10, 30)] + [(20, x) for x in range(50, 64)],  # two rows
        [(47, x) for x in range(0, 64)],                      # bottom edge
    ]
    for sp in spreads:
        for (z, x) in sp:
            rec_iz.append(z)
            rec_ix.append(x)
        ptr.append(len(rec_iz))
    geom = Geometry(src_iz=np.array([2, 0, 30, 10, 47], np.int32),
                    src_ix=np.array([5, 0, 33, 63, 20], np.int32),
                    rec_ptr=np.array(ptr, np.int32), rec_iz=np.array(rec_iz, np.int32),
                    rec_ix=np.array(rec_ix, np.int32), nt=np.array([300, 170, 2, 251, 90], np.int32))
    grid = Grid(nz, nx, 10.0, 1e-3, 300, 12, 2300.0)
    v_true = gaussian_anomaly(nz, nx, 2000.0, 0.15, 6.0, iz0=20, ix0=30)
    v_start = gaussian_anomaly(nz, nx, 2000.0, 0.05, 9.0, iz0=24, ix0=34)
    # per-shot wavelets of different peak frequency
    wav = np.stack([ricker(f, 1e-3, 300) for f in (12.0, 15.0, 10.0, 18.0, 20.0)]).astype(np.float32)
    return grid, geom, v_true, v_start, wav


# ------------------------------------------------------------------ forward
@pytest.mark.parametrize("name", list(EXECS))
def test_forward_tiny(name):
    w = tiny_24x16(nt=300)
    ref = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    got = cpu(B.forward(w.v_true, w.wavelet, w.grid, w.geom, EXECS[name]))
    assert report(f"forward tiny {name}", rel(got, ref), TRACE_TOL) < TRACE_TOL


@pytest.mark.parametrize("name", list(EXECS))
def test_forward_ragged(name):
    grid, geom, v_true, _, wav = ragged_geometry()
    ref = oracle.forward_traces(v_true, grid, geom, wav)
    got = cpu(B.forward(v_true, wav, grid, geom, EXECS[name]))
    for s in range(geom.nshot):
        a, b = geom.rec_ptr[s], geom.rec_ptr[s + 1]
        if b > a and np.any(ref[a:b] != 0):
            assert report(f"forward ragged {name} shot {s}", rel(got[a:b], ref[a:b]), TRACE_TOL) < TRACE_TOL
    assert np.all(got[:, 0] == 0)
    for s in range(geom.nshot):
        a, b = geom.rec_ptr[s], geom.rec_ptr[s + 1]
        assert np.all(got[a:b, geom.nt[s]:] == 0)


def test_forward_anomaly_full():
    w = anomaly_200x100()
    ref = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    got = cpu(B.forward(w.v_true, w.wavelet, w.grid, w.geom))
    assert report("forward anomaly 200x100", rel(got, ref), TRACE_TOL) < TRACE_TOL


# ------------------------------------------------------------------ gradient
@pytest.fixture(scope="module")
def anomaly_ref():
    w = anomaly_200x100()
    d_obs = oracle.forward_traces(w.v_true, w.grid, w.geom, w.wavelet)
    out = {}
    for kind in ("int", "l2"):
        J, g, H1, E = oracle.gradient(w.v_start, w.grid, w.geom, w.wavelet, d_obs, kind, return_parts=True)
        out[kind] = (J, g, H1, E)
    out["syn"] = oracle.forward_traces(w.v_start, w.grid, w.geom, w.wavelet)
    return w, d_obs, out


@pytest.mark.parametrize("kind", ["int", "l2"])
def test_gradient_anomaly_full(anomaly_ref, kind):
    w, d_obs, ref = anomaly_ref
    J, g, H1, _ = ref[kind]
    Jg, gg, Hg, _ = B.gradient(w.v_start, w.wavelet, w.grid, w.geom, d_obs.astype(np.float32), kind)
    jt = j_tolerance(ref["syn"], d_obs, kind, w.grid.dt)
    assert report(f"J anomaly {kind}", abs(float(Jg) - J) / J, jt) <= jt
    assert report(f"grad anomaly {kind}", rel(cpu(gg), g), GRAD_TOL) < GRAD_TOL
    assert report(f"H1 anomaly {kind}", rel(cpu(Hg), H1), GRAD_TOL) < GRAD_TOL


@pytest.mark.parametrize("rcv", ["pm", "none"])
def test_offset_diagonal_anomaly_full(anomaly_ref, rcv):
    w, d_obs, ref = anomaly_ref
    _, _, _, E = ref["int"]
    H = 4
    A = [oracle.aperture_factor(w.grid, *w.geom.shot(s)[2:4], model=rcv) for s in range(w.geom.nshot)]
    Dref = oracle.offset_diag(w.v_start, E, A, H)
    _, _, _, Dg = B.gradient(w.v_start, w.wavelet, w.grid, w.geom, d_obs.astype(np.float32), "int", hmax=H,
                             rcv_model=rcv)
    Dg = cpu(Dg)
    for h in range(2 * H + 1):
        assert report(f"D anomaly {rcv} h={h - H}", rel(Dg[h], Dref[h]), GRAD_TOL) < GRAD_TOL, h


def test_hessian_diag_forward_only(anomaly_ref):
    w, _, ref = anomaly_ref
    _, _, H1, E = ref["int"]
    got = cpu(B.hessian_diag(w.v_start, w.wavelet, w.grid, w.geom, B.HESS_EQ1))
    assert report("H1 forward-only", rel(got, H1), GRAD_TOL) < GRAD_TOL
    H = 3
    A = [oracle.aperture_factor(w.grid, *w.geom.shot(0)[2:4])]
    Dref = oracle.offset_diag(w.v_start, E, A, H)
    Dg = cpu(B.hessian_diag(w.v_start, w.wavelet, w.grid, w.geom, B.HESS_OFFSET, hmax=H))
    assert report("D forward-only", rel(Dg, Dref), GRAD_TOL) < GRAD_TOL


@pytest.mark.parametrize("name", list(EXECS))
@pytest.mark.parametrize("kind", ["int", "l2"])
def test_gradient_ragged(name, kind):
    grid, geom, v_true, v_start, wav = ragged_geometry()
    d_obs = oracle.forward_traces(v_true, grid, geom, wav)
    J, g, H1, E = oracle.gradient(v_start, grid, geom, wav, d_obs, kind, return_parts=True)
    H = 2
    A = [oracle.aperture_factor(grid, *geom.shot(s)[2:4]) if geom.rec_ptr[s + 1] > geom.rec_ptr[s]
         else np.zeros((grid.nz, grid.nx)) for s in range(geom.nshot)]
    Dref = oracle.offset_diag(v_start, E, A, H)
    Jg, gg, Hg, Dg = B.gradient(v_start, wav, grid, geom, d_obs.astype(np.float32), kind, EXECS[name], hmax=H)
    syn = oracle.forward_traces(v_start, grid, geom, wav)
    jt = j_tolerance(syn, d_obs, kind, grid.dt)
    tag = f"ragged {kind} {name}"
    assert report(f"J {tag}", abs(float(Jg) - J) / J, jt) <= jt
    assert report(f"grad {tag}", rel(cpu(gg), g), GRAD_TOL) < GRAD_TOL
    assert report(f"H1 {tag}", rel(cpu(Hg), H1), GRAD_TOL) < GRAD_TOL
    assert report(f"D {tag}", rel(cpu(Dg), Dref), GRAD_TOL) < GRAD_TOL


def test_gradient_is_deterministic():
    grid, geom, v_true, v_start, wav = ragged_geometry()
    d_obs = random_traces(geom, grid.nt_max, seed=5, scale=1e-3)
    ex = EXECS["batched_graph"]
    a = B.gradient(v_start, wav, grid, geom, d_obs, "int", ex, hmax=2)
    b = B.gradient(v_start, wav, grid, geom, d_obs, "int", ex, hmax=2)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("call", ["gradient", "extended_image", "autograd"])
def test_launch_chains_give_the_same_bits(call):
    """Graph chunks split into 2, 3 or 4 independent launch chains over shares
    of the shots (ragged case, 5 shots: shares of 2/3, 1/2/2, 1/1/1/2) give
    the bits of one chain: the split changes which launch a shot's work runs
    in, not the order of any sum."""
    from paper_1406_1864_amd.autograd import FWIProblem, fwi_misfit
    grid, geom, v_true, v_start, wav = ragged_geometry()
    d_obs = random_traces(geom, grid.nt_max, seed=7, scale=1e-3)
    outs = []
    for nb in (1, 2, 3, 4):
        ex = B.make_exec(shots_in_flight=5, shots_in_flight_reverse=5, tile_rows=16, tile_rows_reverse=8,
                         graph_steps=3, reverse_steps=2, forward_steps=2, graph_branches=nb)
        if call == "gradient":
            outs.append(B.gradient(v_start, wav, grid, geom, d_obs, "int", ex, hmax=2))
        elif call == "extended_image":
            outs.append(B.extended_image(v_start, wav, grid, geom, d_obs, 2, "int", ex))
        else:
            pr = FWIProblem(grid, geom, wav, d_obs, "int", ex, hmax=2)
            v = torch.tensor(v_start, device="cuda", requires_grad=True)
            J = fwi_misfit(v, pr)
            J.backward()
            outs.append((J.detach(), v.grad, pr.illum, pr.offset))
    for nb, o in zip((2, 3, 4), outs[1:]):
        for k, (x, y) in enumerate(zip(outs[0], o)):
            assert torch.equal(x, y), (call, nb, k)


def test_calls_from_two_threads_on_two_streams():
    """Two host threads call fwi_gradient at the same time, each on a stream and
    a workspace of its own (both capture their graph chunks in that call):
    each result has the bits of the same call made alone."""
    import threading
    grid, geom, v_true, v_start, wav = ragged_geometry()
    d_obs = random_traces(geom, grid.nt_max, seed=9, scale=1e-3)
    ex = B.make_exec(shots_in_flight=5, tile_rows=16, tile_rows_reverse=16, graph_steps=4, reverse_steps=2,
                     forward_steps=2)
    ref = B.gradient(v_start, wav, grid, geom, d_obs, "int", ex, hmax=2)
    torch.cuda.synchronize()
    out, errors = [None, None], []
    start = threading.Barrier(2)

    def work(i):
        try:
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                start.wait(timeout=60)
                out[i] = B.gradient(v_start, wav, grid, geom, d_obs, "int", ex, hmax=2)
            stream.synchronize()
        except Exception as e:  # reported in the main thread
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,), daemon=True) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    for o in out:
        assert o is not None
        for x, y in zip(ref, o):
            assert torch.equal(x, y)


def test_no_shots_gives_zero():
    grid, geom, v_true, v_start, wav = ragged_geometry()
    empty = Geometry(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(1, np.int32), np.zeros(0, np.int32),
                     np.zeros(0, np.int32), np.zeros(0, np.int32))
    J, g, H1, D = B.gradient(v_start, wav[0], grid, empty, np.zeros((1, grid.nt_max), np.float32), "int", hmax=1)
    assert float(J) == 0.0
    assert float(g.abs().max()) == 0.0 and float(H1.abs().max()) == 0.0 and float(D.abs().max()) == 0.0


def test_nonfinite_velocity_is_flagged():
    w = tiny_24x16(nt=50)
    v = w.v_start.copy()
    v[3, 4] = np.nan
    ws = B.workspace(w.grid, w.geom, B.WS_FORWARD)
    data = torch.empty((w.geom.ntrace, w.grid.nt_max), device="cuda")
    vd = torch.as_tensor(v, device="cuda")
    wd = torch.as_tensor(w.wavelet, device="cuda")
    B.fwi_forward(w.grid, w.geom, None, vd, wd, 0, data, ws, ws.numel())
    assert B.fwi_status(ws) == B.FWI_ERR_NONFINITE
    vd = torch.as_tensor(w.v_start, device="cuda")
    B.fwi_forward(w.grid, w.geom, None, vd, wd, 0, data, ws, ws.numel())
    assert B.fwi_status(ws) == B.FWI_OK


# ------------------------------------------------------------------ preconditioner
def test_precondition_matches_oracle(anomaly_ref):
    w, d_obs, ref = anomaly_ref
    J, g, H1, E = ref["int"]
    H = 4
    A = [oracle.aperture_factor(w.grid, *w.geom.shot(0)[2:4])]
    D = oracle.offset_diag(w.v_start, E, A, H)
    v = torch.as_tensor(w.v_start, device="cuda")
    gt = torch.as_tensor(g.astype(np.float32), device="cuda")
    out = B.precondition(v, gt, torch.as_tensor(H1.astype(np.float32), device="cuda"), w.grid, B.PRECOND_SHOT)
    ref_s = oracle.precondition(g.astype(np.float32), oracle.shot_scaling(w.v_start, H1.astype(np.float32)))
    assert report("precondition shot", rel(cpu(out), ref_s), 1e-5) < 1e-5
    out = B.precondition(v, gt, torch.as_tensor(D.astype(np.float32), device="cuda"), w.grid, B.PRECOND_OFFSET,
                         hmax=H)
    ref_o = oracle.precondition(g.astype(np.float32), oracle.offset_scaling(D.astype(np.float32)))
    assert report("precondition offset", rel(cpu(out), ref_o), 1e-5) < 1e-5
