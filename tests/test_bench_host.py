"""Host-side pieces of bench.py: the algorithmic byte model of the reverse
and forward steps, counted cell by cell on a small grid, and the lookup of
the committed counter summaries that supplies `roofline.traffic`."""
import json
import os

import pytest

import bench
from paper_1406_1864_amd.synthetic import Grid


def classify(grid):
    """(model cells, strip-ring cells, other sponge cells) of the padded grid,
    walking every cell: the ring is the 4 cells just outside the model on
    each side, alongside its rows and columns (not the corners)."""
    nz, nx, N = grid.nz, grid.nx, grid.nsponge
    model = ring = other = 0
    for z in range(-N, nz + N):
        for x in range(-N, nx + N):
            zin, xin = 0 <= z < nz, 0 <= x < nx
            if zin and xin:
                model += 1
            elif (xin and (-4 <= z < 0 or nz <= z < nz + 4)) or (zin and (-4 <= x < 0 or nx <= x < nx + 4)):
                ring += 1
            else:
                other += 1
    return model, ring, other


@pytest.mark.parametrize("nz,nx,N", [(12, 20, 6), (7, 9, 4), (30, 11, 10)])
def test_reverse_and_forward_byte_models_count_every_cell(nz, nx, N):
    grid = Grid(nz, nx, 10.0, 1e-3, 100, N, 2000.0)
    model, ring, other = classify(grid)
    nrec = 5
    assert bench.reverse_bytes_per_shot_step(grid, nrec) == 44 * model + 24 * ring + 16 * other + 4 * nrec
    K = 10
    padded = model + ring + other
    assert bench.forward_bytes_per_shot_step(grid, nrec, K) == pytest.approx(
        20 * padded + 4 * ring + 8 * model / K + 4 * nrec)


def summary(tag):
    with open(os.path.join(bench.ROOT, "profiles", f"k_reverse2_pmc_{tag}.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("workload,tag", [("offset", "layered_2048x768"), ("layered", "layered_1024x384")])
def test_measured_traffic_matches_only_the_counted_settings(workload, tag, monkeypatch):
    doc = summary(tag)
    monkeypatch.setattr(bench, "kernel_hash", lambda: doc["kernel_source_sha"])
    chosen = dict(doc["launch_config"])
    assert bench.measured_traffic("k_reverse2", chosen, workload) == doc["bytes_per_launch"]
    # another band height the summary also counted gives that entry's bytes
    other = doc["other_reverse_settings"][0]
    alt = dict(chosen, tile_rows_reverse=other["launch_config"]["tile_rows_reverse"])
    assert bench.measured_traffic("k_reverse2", alt, workload) == other["bytes_per_launch"]
    # settings it did not count, or other kernel source, give none
    for key, value in (("graph_branches", 1), ("prefetch_reverse", 3), ("shots_in_flight_reverse", 7),
                       ("reverse_steps", 1), ("tile_rows_reverse", 13)):
        assert bench.measured_traffic("k_reverse2", dict(chosen, **{key: value}), workload) is None, key
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.measured_traffic("k_reverse2", chosen, workload) is None
    assert bench.measured_traffic("k_reverse2", chosen, "ragged") is None

