"""GPU parity of Born modelling (fwi_born, eq. (4)) and of the Gauss-Newton
Hessian-vector product (fwi_gn_hvp) against the FP64 oracle: Born traces to
the seismogram tolerance (1e-4), H dv to the gradient tolerance (1e-3);
at full grid size the properties <dv, H dv> = 2 J and <a, H b> = <H a, b>."""
import numpy as np
import pytest

import oracle
from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import (Grid, anomaly_200x100, bump_direction, layered_1024x384,
                                           noise_direction, tiny_24x16)

from helpers import GRAD_TOL, TRACE_TOL, rel, report
from test_gpu_parity import EXECS, cpu, ragged_geometry

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def perturbation(nz, nx, seed):
    """A smooth velocity perturbation (m/s) reaching the model edges."""
    rng = np.random.default_rng(seed)
    return (bump_direction(nz, nx, sigma=max(2.0, min(nz, nx) / 6.0)) * 40.0
            + rng.standard_normal((nz, nx)) * 5.0)


@pytest.mark.parametrize("name", list(EXECS))
def test_born_tiny(name):
    w = tiny_24x16(nt=300)
    dv = perturbation(w.grid.nz, w.grid.nx, 1)
    ref = oracle.born(w.v_start, w.grid, w.geom, w.wavelet, dv)
    got = cpu(B.born(w.v_start, w.wavelet, w.grid, w.geom, dv, EXECS[name]))
    assert report(f"born tiny {name}", rel(got, ref), TRACE_TOL) < TRACE_TOL


@pytest.mark.parametrize("name", list(EXECS))
def test_born_ragged(name):
    grid, geom, v_true, v_start, wav = ragged_geometry()
    dv = perturbation(grid.nz, grid.nx, 2)
    ref = oracle.born(v_start, grid, geom, wav, dv)
    got = cpu(B.born(v_start, wav, grid, geom, dv, EXECS[name]))
    for s in range(geom.nshot):
        a, b = geom.rec_ptr[s], geom.rec_ptr[s + 1]
        if b > a and np.any(ref[a:b] != 0):
            assert report(f"born ragged {name} shot {s}", rel(got[a:b], ref[a:b]), TRACE_TOL) < TRACE_TOL
        assert np.all(got[a:b, geom.nt[s]:] == 0)


def check_hvp(tag, ref, got, dv):
    Jb, H = ref
    Jg, Hg = got
    Hg = cpu(Hg)
    assert report(f"gn J {tag}", abs(float(Jg) - Jb) / Jb, TRACE_TOL) <= TRACE_TOL
    assert report(f"gn H dv {tag}", rel(Hg, H), GRAD_TOL) < GRAD_TOL
    # <dv, H dv> = |W J dv|^2 = 2 J, from the same call
    q = float(np.sum(dv.astype(np.float64) * Hg))
    assert report(f"gn <dv,Hdv>/2J {tag}", abs(q / (2.0 * float(Jg)) - 1.0), GRAD_TOL) < GRAD_TOL


@pytest.mark.parametrize("name", list(EXECS))
@pytest.mark.parametrize("kind", ["int", "l2"])
def test_gn_hvp_tiny(name, kind):
    w = tiny_24x16(nt=300)
    dv = perturbation(w.grid.nz, w.grid.nx, 3)
    ref = oracle.gn_hvp(w.v_start, w.grid, w.geom, w.wavelet, dv, kind)
    got = B.gn_hvp(w.v_start, w.wavelet, w.grid, w.geom, dv, kind, EXECS[name])
    check_hvp(f"tiny {kind} {name}", ref, got, dv)


@pytest.mark.parametrize("name", list(EXECS))
def test_gn_hvp_ragged(name):
    grid, geom, v_true, v_start, wav = ragged_geometry()
    dv = perturbation(grid.nz, grid.nx, 4)
    ref = oracle.gn_hvp(v_start, grid, geom, wav, dv, "int")
    got = B.gn_hvp(v_start, wav, grid, geom, dv, "int", EXECS[name])
    check_hvp(f"ragged {name}", ref, got, dv)


def test_gn_hvp_anomaly_full():
    w = anomaly_200x100()
    dv = perturbation(w.grid.nz, w.grid.nx, 5)
    ref = oracle.gn_hvp(w.v_start, w.grid, w.geom, w.wavelet, dv, "int")
    got = B.gn_hvp(w.v_start, w.wavelet, w.grid, w.geom, dv, "int")
    check_hvp("anomaly 200x100", ref, got, dv)


def test_gn_hvp_layered_full_size_properties():
    """1024x384, 8 shots, nt 400, batched with graph chunks: H is symmetric
    positive semi-definite, <a, H b> = <H a, b> and <a, H a> = 2 J(a)."""
    w = layered_1024x384(nshot=64)
    geom = w.geom.subset(list(range(0, 64, 8))).with_nt(400)
    grid = Grid(w.grid.nz, w.grid.nx, w.grid.dx, w.grid.dt, 400, w.grid.nsponge, w.grid.v_ref)
    wav = w.wavelet[:400]
    a = bump_direction(grid.nz, grid.nx) * 50.0
    b = noise_direction(grid.nz, grid.nx) * 50.0
    ex = B.make_exec(shots_in_flight=8, tile_rows=16, graph_steps=32)
    Ja, Ha = B.gn_hvp(w.v_start, wav, grid, geom, a, "int", ex)
    Jb, Hb = B.gn_hvp(w.v_start, wav, grid, geom, b, "int", ex)
    Ha, Hb = cpu(Ha).astype(np.float64), cpu(Hb).astype(np.float64)
    aHb, bHa = float(np.sum(a * Hb)), float(np.sum(b * Ha))
    assert report("gn layered symmetry", abs(aHb - bHa) / abs(aHb), GRAD_TOL) < GRAD_TOL
    for tag, d, J, H in (("a", a, Ja, Ha), ("b", b, Jb, Hb)):
        q = float(np.sum(d * H))
        assert q > 0
        assert report(f"gn layered <{tag},H{tag}>/2J", abs(q / (2.0 * float(J)) - 1.0), GRAD_TOL) < GRAD_TOL
    # the Born data of the same perturbation give the same J
    dd = cpu(B.born(w.v_start, wav, grid, geom, a, ex)).astype(np.float64)
    R = grid.dt * np.cumsum(dd, axis=-1)
    assert report("gn layered J vs Born data", abs(0.5 * np.sum(R * R) / float(Ja) - 1.0), TRACE_TOL) < TRACE_TOL
