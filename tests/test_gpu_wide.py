"""GPU parity on a grid several workgroups wide, cell by cell.

The two-step sweeps (k_forward2, k_reverse2) tile x in workgroups of 248
owned columns with a 4-column halo recomputed by the first step, and the
one-step sweeps in 64-column wavefront tiles.  Here the padded grid is 600
columns wide (model 560 + 2 x 20 sponge), so the two-step tiling has three
workgroups and the inter-workgroup halo exchange runs in every launch mode;
sources sit beside the workgroup boundaries (model columns 228 and 476) and
the records are long enough for the wavefields to cross them.

Every output is compared with the FP64 oracle on every cell: relative L2
over the whole array, the largest element-wise deviation relative to the
largest reference magnitude, and the relative L2 of every model column (an
error confined to the few columns beside a workgroup boundary moves the
last of these by orders of magnitude more than the first).
"""
import multiprocessing

import numpy as np
import pytest

from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import random_traces

from helpers import GRAD_TOL, TRACE_TOL, J_TOL, max_rel, rel, report
from test_gpu_parity import EXECS, cpu
from wide_case import HMAX, oracle_shot, wide_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# model columns where the two-step tiling's workgroups meet (padded 248, 496)
WG_EDGES = (228, 476)


@pytest.fixture(scope="module")
def wide_ref():
    """Recorded data: seeded noise at 0.3 x the RMS of each shot's modelled
    traces (a residual at every receiver and sample, so that the adjoint
    wavefield fills the model); the oracle runs one process per shot."""
    grid, geom, v, wav = wide_case()
    with multiprocessing.get_context("spawn").Pool(geom.nshot) as pool:
        parts = pool.map(oracle_shot, range(geom.nshot))
    ref = {k: sum(p[k] for p in parts) for k in ("J", "g", "H1", "D", "Je", "I")}
    ref["syn"] = np.concatenate([p["syn"] for p in parts])
    d_obs = np.concatenate([p["d_obs"] for p in parts]).astype(np.float32)
    return (grid, geom, v, wav, d_obs), ref


def columns(tag, got, ref, tol):
    """Relative L2 of every model column (last axis) of a [.., nz, nx] array,
    for the columns whose reference is not negligible."""
    got = np.asarray(got, np.float64).reshape(-1, got.shape[-1])
    ref = np.asarray(ref, np.float64).reshape(-1, ref.shape[-1])
    num = np.linalg.norm(got - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    live = den > 1e-3 * den.max()
    err = num[live] / den[live]
    worst = int(np.flatnonzero(live)[np.argmax(err)])
    near = [x for e in WG_EDGES for x in range(e - 6, e + 6) if live[x]]
    edge = float(np.max(num[near] / den[near]))
    assert report(f"{tag} per column (worst x={worst})", float(err.max()), tol) < tol
    assert report(f"{tag} per column beside workgroup edges", edge, tol) < tol


def compare(tag, got, ref, tol):
    assert report(f"{tag} rel L2", rel(got, ref), tol) < tol
    assert report(f"{tag} max element", max_rel(got, ref), tol) < tol


@pytest.mark.parametrize("name", list(EXECS))
def test_wide_forward(wide_ref, name):
    (grid, geom, v, wav, _), ref = wide_ref
    got = cpu(B.forward(v, wav, grid, geom, EXECS[name]))
    for s in range(geom.nshot):
        a, b = geom.rec_ptr[s], geom.rec_ptr[s + 1]
        compare(f"wide traces {name} shot {s}", got[a:b], ref["syn"][a:b], TRACE_TOL)
        assert np.all(got[a:b, geom.nt[s]:] == 0)


@pytest.mark.parametrize("name", list(EXECS))
def test_wide_gradient(wide_ref, name):
    (grid, geom, v, wav, d_obs), ref = wide_ref
    J, g, H1, D = B.gradient(v, wav, grid, geom, d_obs, "int", EXECS[name], hmax=HMAX)
    tag = f"wide {name}"
    assert report(f"J {tag}", abs(float(J) - ref["J"]) / ref["J"], J_TOL) <= J_TOL
    g, H1, D = cpu(g), cpu(H1), cpu(D)
    compare(f"grad {tag}", g, ref["g"], GRAD_TOL)
    columns(f"grad {tag}", g, ref["g"], GRAD_TOL)
    compare(f"H1 {tag}", H1, ref["H1"], GRAD_TOL)
    columns(f"H1 {tag}", H1, ref["H1"], GRAD_TOL)
    for h in range(2 * HMAX + 1):
        compare(f"D {tag} h={h - HMAX}", D[h], ref["D"][h], GRAD_TOL)
    columns(f"D {tag}", D, ref["D"], GRAD_TOL)


@pytest.mark.parametrize("name", list(EXECS))
def test_wide_extended_image(wide_ref, name):
    (grid, geom, v, wav, d_obs), ref = wide_ref
    J, g, image = B.extended_image(v, wav, grid, geom, d_obs, HMAX, "int", EXECS[name])
    tag = f"wide ext {name}"
    assert report(f"J {tag}", abs(float(J) - ref["Je"]) / ref["Je"], J_TOL) <= J_TOL
    image = cpu(image)
    for h in range(2 * HMAX + 1):
        compare(f"image {tag} h={h - HMAX}", image[h], ref["I"][h], GRAD_TOL)
    columns(f"image {tag}", image, ref["I"], GRAD_TOL)


@pytest.mark.parametrize("call", ["gradient", "extended_image"])
def test_wide_launch_chains_give_the_same_bits(call):
    """Three two-step workgroups wide: graph chunks in 2 and 3 independent
    launch chains (shares of 1 + 2 and 1 + 1 + 1 of the 3 shots) give the
    bits of one chain."""
    grid, geom, v, wav = wide_case()
    d_obs = random_traces(geom, grid.nt_max, seed=77, scale=1e-3)
    outs = []
    for nb in (1, 2, 3):
        ex = B.make_exec(shots_in_flight=3, tile_rows=32, tile_rows_reverse=24, graph_steps=8, reverse_steps=2,
                         forward_steps=2, graph_branches=nb)
        if call == "gradient":
            outs.append(B.gradient(v, wav, grid, geom, d_obs, "int", ex, hmax=HMAX))
        else:
            outs.append(B.extended_image(v, wav, grid, geom, d_obs, HMAX, "int", ex))
    for nb, o in zip((2, 3), outs[1:]):
        for k, (x, y) in enumerate(zip(outs[0], o)):
            assert torch.equal(x, y), (call, nb, k)
