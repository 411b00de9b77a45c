"""FP64 CPU oracle for the preconditioned FWI gradient.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``; never by the product path.  It
shares no code with the HIP implementation.
"""
from .acoustic import (C8, CFL_LIMIT, Propagator, laplacian, sponge_gamma, padded_q,
                       forward, forward_traces, misfit, misfit_l2, misfit_time_integral,
                       adjoint, source_adjoint, shot_gradient, imaging, gradient, illumination,
                       gradient_eq3_literal, end_of_record_term)
from .hessian import (aperture_factor, offset_diag, shot_scaling, offset_scaling,
                      precondition, extended_born_columns, offset_diag_exact, extended_image,
                      born_shot, born, gn_hvp, spectral_bins, green_series,
                      source_series, power, offset_diag_spectral, offset_diag_spectral_cells)
