"""Host-side checks of the C ABI (no GPU needed, no compute call).

The library must load, export every function include/fwi.h declares, and
reject bad input with the documented error code before it touches the GPU
(every check below returns before any HIP call is made).
"""
import ctypes

import numpy as np
import pytest

from paper_1406_1864_amd import binding as B
from paper_1406_1864_amd.synthetic import (Grid, Geometry, tiny_24x16, layered_1024x384, offset_2048x768,
                                           ragged_1024x384)


@pytest.fixture(scope="module")
def lib():
    return B.load()


def test_exports_every_declared_symbol(lib):
    names = B.header_functions()
    assert len(names) >= 10, names
    for n in names:
        assert hasattr(lib, n), n


def _tiny():
    w = tiny_24x16(nt=64)
    return w.grid, w.geom


def test_validate_ok(lib):
    g, geo = _tiny()
    assert B.fwi_validate(g, geo) == B.FWI_OK


@pytest.mark.parametrize("mutate,code", [
    (lambda g, geo: setattr(g, "v_ref", 6000.0), B.FWI_ERR_CFL),
    (lambda g, geo: setattr(g, "nsponge", 3), B.FWI_ERR_ARG),
    (lambda g, geo: setattr(g, "dt", 0.0), B.FWI_ERR_ARG),
    (lambda g, geo: setattr(g, "nt_max", 1), B.FWI_ERR_ARG),
    (lambda g, geo: geo.src_ix.__setitem__(0, 24), B.FWI_ERR_GEOM),
    (lambda g, geo: geo.src_iz.__setitem__(1, -1), B.FWI_ERR_GEOM),
    (lambda g, geo: geo.rec_ix.__setitem__(3, 99), B.FWI_ERR_GEOM),
    (lambda g, geo: geo.rec_ix.__setitem__(1, geo.rec_ix[0]), B.FWI_ERR_GEOM),
    (lambda g, geo: geo.nt.__setitem__(0, 65), B.FWI_ERR_GEOM),
    (lambda g, geo: geo.nt.__setitem__(0, 1), B.FWI_ERR_GEOM),
    (lambda g, geo: geo.rec_ptr.__setitem__(1, 7), B.FWI_ERR_GEOM),
])
def test_validate_rejects(lib, mutate, code):
    g, geo = _tiny()
    mutate(g, geo)
    assert B.fwi_validate(g, geo) == code
    assert len(B.last_error()) > 0


def test_cfl_bound_matches_scheme():
    import oracle
    assert abs(B.FWI_CFL_LIMIT - oracle.CFL_LIMIT) < 1e-15
    g, geo = _tiny()
    g.v_ref = 0.999 * B.FWI_CFL_LIMIT * g.dx / g.dt
    assert B.fwi_validate(g, geo) == B.FWI_OK
    g.v_ref = 1.001 * B.FWI_CFL_LIMIT * g.dx / g.dt
    assert B.fwi_validate(g, geo) == B.FWI_ERR_CFL


def test_workspace_sizes(lib):
    g, geo = _tiny()
    fwd = B.fwi_workspace_bytes(g, geo, None, B.WS_FORWARD)
    grad = B.fwi_workspace_bytes(g, geo, None, B.WS_GRADIENT)
    auto = B.fwi_workspace_bytes(g, geo, None, B.WS_AUTOGRAD)
    hess = B.fwi_workspace_bytes(g, geo, None, B.WS_HESSIAN)
    assert 0 < fwd < hess < grad <= auto
    assert B.fwi_workspace_bytes(g, geo, None, B.WS_PRECOND) >= 4
    g.v_ref = 1e5
    assert B.fwi_workspace_bytes(g, geo, None, B.WS_GRADIENT) == 0


def test_workspace_fits_an_mi355x_at_full_sizes(lib):
    """The checkpoints of the batched gradient fit in 288 GB of HBM."""
    for w in (layered_1024x384(), ragged_1024x384()):
        ex = B.make_exec(shots_in_flight=64)
        n = B.fwi_workspace_bytes(w.grid, w.geom, ex, B.WS_GRADIENT)
        assert 0 < n < 200e9, (w.name, n)


def test_entry_points_reject_before_launch(lib):
    """Bad arguments come back as error codes with no HIP call (fake device
    pointers are never dereferenced)."""
    g, geo = _tiny()
    fake = 0x1000
    with pytest.raises(B.FwiError) as e:
        B.fwi_forward(g, geo, None, fake, fake, 0, fake, fake, 16, stream=0)
    assert e.value.code == B.FWI_ERR_WORKSPACE
    with pytest.raises(B.FwiError) as e:
        B.fwi_gradient(g, geo, None, fake, fake, 0, fake, "int", fake, fake, None, 0, "pm", None, fake, 16,
                       stream=0)
    assert e.value.code == B.FWI_ERR_WORKSPACE
    with pytest.raises(B.FwiError) as e:
        B.fwi_gradient(g, geo, None, fake, fake, 0, fake, "int", fake, fake, None, 99, "pm", fake, fake, 1 << 40,
                       stream=0)
    assert e.value.code == B.FWI_ERR_ARG
    with pytest.raises(B.FwiError) as e:
        B.fwi_forward(g, geo, None, fake, fake, 7, fake, fake, 1 << 40, stream=0)
    assert e.value.code == B.FWI_ERR_ARG
    g.v_ref = 1e5
    with pytest.raises(B.FwiError) as e:
        B.fwi_hessian_diag(g, geo, None, fake, fake, 0, B.HESS_EQ1, 0, "pm", fake, fake, 1 << 40, stream=0)
    assert e.value.code == B.FWI_ERR_CFL
    g, geo = _tiny()
    with pytest.raises(B.FwiError) as e:
        B.fwi_misfit_backward(g, geo, None, fake, fake, 0, None, fake, None, 0, "pm", None, fake, 1 << 40,
                              stream=0)
    assert e.value.code == B.FWI_ERR_STATE
    with pytest.raises(B.FwiError) as e:
        B.fwi_precondition(g, fake, fake, 5, fake, 0, 0.01, fake, fake, 256, stream=0)
    assert e.value.code == B.FWI_ERR_ARG


def test_extended_image_sizing_and_rejects(lib):
    """The extended image's workspace adds its lam/D rings and offset sums to
    the gradient's; out-of-range offsets and a missing output are rejected
    before any HIP call."""
    g, geo = _tiny()
    grad = B.fwi_workspace_bytes(g, geo, None, B.WS_GRADIENT)
    e4 = B.fwi_workspace_bytes(g, geo, None, B.WS_EXTIMAGE, 4)
    e8 = B.fwi_workspace_bytes(g, geo, None, B.WS_EXTIMAGE, 8)
    assert grad < e4 < e8
    assert B.fwi_workspace_bytes(g, geo, None, B.WS_EXTIMAGE, 33) == 0
    assert B.fwi_workspace_bytes(g, geo, None, B.WS_EXTIMAGE, -1) == 0
    assert B.fwi_workspace_bytes(g, geo, None, B.WS_EXTIMAGE, 24) == 0   # hmax must be < nx
    q = B.fwi_exec_query(g, geo, None, B.WS_EXTIMAGE)
    assert q["graph_steps"] > 0
    fake = 0x1000
    with pytest.raises(B.FwiError) as e:
        B.fwi_extended_image(g, geo, None, fake, fake, 0, fake, "int", fake, None, 4, None, fake, 1 << 40, stream=0)
    assert e.value.code == B.FWI_ERR_ARG
    with pytest.raises(B.FwiError) as e:
        B.fwi_extended_image(g, geo, None, fake, fake, 0, fake, "int", fake, None, 40, fake, fake, 1 << 40, stream=0)
    assert e.value.code == B.FWI_ERR_ARG
    with pytest.raises(B.FwiError) as e:
        B.fwi_extended_image(g, geo, None, fake, fake, 0, fake, "int", fake, None, 4, fake, fake, 16, stream=0)
    assert e.value.code == B.FWI_ERR_WORKSPACE


def test_eq3_literal_is_gradient_only(lib):
    """FWI_MISFIT_EQ3_LITERAL is not the gradient of J: the autograd pair and
    the extended image refuse it before any HIP call."""
    g, geo = _tiny()
    fake = 0x1000
    with pytest.raises(B.FwiError) as e:
        B.fwi_misfit_forward(g, geo, None, fake, fake, 0, fake, "eq3", fake, fake, 1 << 40, stream=0)
    assert e.value.code == B.FWI_ERR_ARG
    with pytest.raises(B.FwiError) as e:
        B.fwi_extended_image(g, geo, None, fake, fake, 0, fake, "eq3", fake, None, 4, fake, fake, 1 << 40, stream=0)
    assert e.value.code == B.FWI_ERR_ARG


def test_reverse_launch_settings(lib):
    """The reverse sweep's shots in flight must divide the forward's, else the
    forward's value is used (the autograd pair: any value up to the number of
    shots); its tile rows default to the forward's."""
    w = layered_1024x384(nshot=8)
    q = B.fwi_exec_query(w.grid, w.geom, B.make_exec(shots_in_flight=8, shots_in_flight_reverse=4,
                                                     tile_rows=32, tile_rows_reverse=12), B.WS_GRADIENT)
    assert (q["shots_in_flight"], q["shots_in_flight_reverse"], q["tile_rows"], q["tile_rows_reverse"]) == \
        (8, 4, 32, 12)
    q = B.fwi_exec_query(w.grid, w.geom, B.make_exec(shots_in_flight=8, shots_in_flight_reverse=3), B.WS_GRADIENT)
    assert q["shots_in_flight_reverse"] == 8
    q = B.fwi_exec_query(w.grid, w.geom, B.make_exec(shots_in_flight=8, tile_rows=16), B.WS_GRADIENT)
    assert q["tile_rows_reverse"] == 16
    # the autograd pair keeps every shot's checkpoints: its reverse sweep groups
    # the shots on its own, up to all of them, whatever the forward batch
    for what, want in ((B.WS_AUTOGRAD, 8), (B.WS_GRADIENT, 2)):
        q = B.fwi_exec_query(w.grid, w.geom, B.make_exec(shots_in_flight=2, shots_in_flight_reverse=8), what)
        assert q["shots_in_flight_reverse"] == want
    q = B.fwi_exec_query(w.grid, w.geom, B.make_exec(shots_in_flight=2, shots_in_flight_reverse=3), B.WS_AUTOGRAD)
    assert q["shots_in_flight_reverse"] == 3
    q = B.fwi_exec_query(w.grid, w.geom, B.make_exec(shots_in_flight=2, shots_in_flight_reverse=99), B.WS_AUTOGRAD)
    assert q["shots_in_flight_reverse"] == 8
    # two forward steps per launch: the gradient's forward sweep only
    for what, want in ((B.WS_GRADIENT, 2), (B.WS_AUTOGRAD, 2), (B.WS_EXTIMAGE, 2), (B.WS_FORWARD, 1),
                       (B.WS_BORN, 1), (B.WS_GNHVP, 1), (B.WS_HESSIAN, 1)):
        assert B.fwi_exec_query(w.grid, w.geom, B.make_exec(forward_steps=2), what)["forward_steps"] == want, what
    assert B.fwi_exec_query(w.grid, w.geom, B.make_exec(forward_steps=2, mode=B.EXEC_PLAIN),
                            B.WS_GRADIENT)["forward_steps"] == 1
    with pytest.raises(B.FwiError):
        B.fwi_exec_query(w.grid, w.geom, B.make_exec(forward_steps=3), B.WS_GRADIENT)
    # independent launch chains per captured chunk: two unless set, one in plain mode
    assert B.fwi_exec_query(w.grid, w.geom, B.make_exec(), B.WS_AUTOGRAD)["graph_branches"] == 2
    for n in (1, 3, 4):
        assert B.fwi_exec_query(w.grid, w.geom, B.make_exec(graph_branches=n), B.WS_AUTOGRAD)["graph_branches"] == n
    assert B.fwi_exec_query(w.grid, w.geom, B.make_exec(mode=B.EXEC_PLAIN), B.WS_GRADIENT)["graph_branches"] == 1
    for bad in (-1, 5):
        with pytest.raises(B.FwiError):
            B.fwi_exec_query(w.grid, w.geom, B.make_exec(graph_branches=bad), B.WS_GRADIENT)
    a = B.fwi_workspace_bytes(w.grid, w.geom, B.make_exec(forward_steps=2), B.WS_GRADIENT)
    b = B.fwi_workspace_bytes(w.grid, w.geom, B.make_exec(forward_steps=1), B.WS_GRADIENT)
    assert a > b                          # two sets of wavefield levels
    g, geo = _tiny()
    with pytest.raises(B.FwiError) as e:
        B.fwi_exec_query(g, geo, B.make_exec(tile_rows_reverse=4), B.WS_GRADIENT)
    a = B.fwi_workspace_bytes(g, geo, B.make_exec(shots_in_flight=2, shots_in_flight_reverse=1), B.WS_GRADIENT)
    b = B.fwi_workspace_bytes(g, geo, B.make_exec(shots_in_flight=2), B.WS_GRADIENT)
    assert 0 < a < b                      # adjoint fields for one reverse slot instead of two


def test_offset_diag_exact_sizing_and_rejects(lib):
    """The exact offset diagonal's workspace grows with the band and the runs
    in flight; bad offsets, a negative band, a free surface, a missing output
    and a short workspace are rejected before any HIP call."""
    w = tiny_24x16(nt=300)      # 301 bins: three 256-column tiles of the DFT matrix; 40 Hz: 25 bins, one tile
    g, geo = w.grid, w.geom
    full = B.fwi_offset_diag_exact_workspace_bytes(g, geo, None, 4, 0.0)
    band = B.fwi_offset_diag_exact_workspace_bytes(g, geo, None, 4, 40.0)
    one = B.fwi_offset_diag_exact_workspace_bytes(g, geo, B.make_exec(shots_in_flight=1), 4, 0.0)
    assert 0 < band < full and 0 < one < full
    # both arithmetics capture FP32 series (the split happens on their way into LDS)
    assert B.fwi_offset_diag_exact_workspace_bytes(g, geo, None, 4, 0.0, B.DFT_BF16X3) == full
    for hmax, fmax, dft in ((33, 0.0, 0), (-1, 0.0, 0), (24, 0.0, 0), (4, -1.0, 0), (4, float("nan"), 0),
                            (4, 0.0, 2)):
        assert B.fwi_offset_diag_exact_workspace_bytes(g, geo, None, hmax, fmax, dft) == 0, (hmax, fmax, dft)
    fake = 0x1000
    with pytest.raises(B.FwiError) as e:
        B.fwi_offset_diag_exact(g, geo, None, fake, fake, 0, 4, 0.0, 0, None, fake, 1 << 40, stream=0)
    assert e.value.code == B.FWI_ERR_ARG
    with pytest.raises(B.FwiError) as e:
        B.fwi_offset_diag_exact(g, geo, None, fake, fake, 0, 40, 0.0, 0, fake, fake, 1 << 40, stream=0)
    assert e.value.code == B.FWI_ERR_ARG
    with pytest.raises(B.FwiError) as e:
        B.fwi_offset_diag_exact(g, geo, None, fake, fake, 0, 4, 0.0, 0, fake, fake, full - 1, stream=0)
    assert e.value.code == B.FWI_ERR_WORKSPACE
    with pytest.raises(B.FwiError) as e:
        B.fwi_offset_diag_exact(g, geo, None, fake, fake, 0, 4, 0.0, 3, fake, fake, 1 << 40, stream=0)
    assert e.value.code == B.FWI_ERR_ARG
    long = Grid(g.nz, g.nx, g.dx, g.dt, 70000, g.nsponge, g.v_ref)
    lgeo = Geometry(geo.src_iz, geo.src_ix, geo.rec_ptr, geo.rec_iz, geo.rec_ix, np.full(2, 70000, np.int32))
    assert B.fwi_offset_diag_exact_workspace_bytes(long, lgeo, None, 4, 0.0) == 0       # 70001 bins
    assert B.fwi_offset_diag_exact_workspace_bytes(long, lgeo, None, 4, 60.0) > 0       # 8401 bins
    g.free_surface = True
    assert B.fwi_offset_diag_exact_workspace_bytes(g, geo, None, 4, 0.0) == 0
    with pytest.raises(B.FwiError) as e:
        B.fwi_offset_diag_exact(g, geo, None, fake, fake, 0, 4, 0.0, 0, fake, fake, 1 << 40, stream=0)
    assert e.value.code == B.FWI_ERR_ARG


def test_offset_diag_exact_fits_an_mi355x_at_full_size(lib):
    """2048x768, nt 8000, band to 60 Hz, the default 4 runs in flight and 8:
    the captured chunks and the spectra fit in 288 GB."""
    w = offset_2048x768()
    for ex in (None, B.make_exec(shots_in_flight=8)):
        for dft in (B.DFT_FP32, B.DFT_BF16X3):
            n = B.fwi_offset_diag_exact_workspace_bytes(w.grid, w.geom, ex, 16, 60.0, dft)
            assert 0 < n < 150e9, (dft, n)


def test_gradient_static_rejects_before_any_hip_call(lib):
    """fwi_gradient_static checks its inputs and its scratch need on the host:
    bad geometry, a bad hmax and a call that needs more than the static
    array's FWI_STATIC_SCRATCH_BYTES are refused before anything touches the
    GPU (here there is none)."""
    fake = 0x1000
    w = layered_1024x384(nshot=4)
    need = B.fwi_workspace_bytes(w.grid, w.geom, B.make_exec(graph_steps=-1), B.WS_GRADIENT, 0)
    assert need > B.FWI_STATIC_SCRATCH_BYTES
    with pytest.raises(B.FwiError) as e:
        B.fwi_gradient_static(w.grid, w.geom, None, fake, fake, 0, fake, "int", fake, fake, None, 0, "pm", None,
                              stream=0)
    assert e.value.code == B.FWI_ERR_WORKSPACE
    g, geo = _tiny()
    bad = Geometry(geo.src_iz, geo.src_ix, geo.rec_ptr, geo.rec_iz, geo.rec_ix + 100, geo.nt)
    with pytest.raises(B.FwiError) as e:
        B.fwi_gradient_static(g, bad, None, fake, fake, 0, fake, "int", fake, fake, None, 0, "pm", None, stream=0)
    assert e.value.code == B.FWI_ERR_GEOM
    with pytest.raises(B.FwiError) as e:
        B.fwi_gradient_static(g, geo, None, fake, fake, 0, fake, "int", fake, fake, None, 40, "pm", fake, stream=0)
    assert e.value.code == B.FWI_ERR_ARG
