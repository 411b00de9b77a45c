"""Shared tolerances and error measures of the GPU parity tests.

Seismograms: relative L2 <= 1e-4; gradients and Hessian diagonals: relative
L2 <= 1e-3 (the accuracy contract of the hot path).  J has no contract of its
own: it is a function of the seismograms, so its tolerance is derived from
the seismogram tolerance.  With W the misfit's data weighting (identity, or
dt times the running sum for eq. (2)) and r = d_syn - d_obs,
|J' - J| <= |<W r, W e>| + |W e|^2 / 2 <= tol |W d_syn| |W r| + ...,
so |dJ| / J <= 2 tol |W d_syn| / |W r| to first order.
"""
import numpy as np

TRACE_TOL = 1e-4
GRAD_TOL = 1e-3


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def weight(x, kind, dt):
    x = np.asarray(x, np.float64)
    return dt * np.cumsum(x, axis=-1) if kind in ("int", 1) else x


def j_tolerance(d_syn, d_obs, kind, dt):
    """Relative tolerance on J implied by TRACE_TOL on the synthetic traces."""
    Wd = weight(d_syn, kind, dt)
    Wr = weight(np.asarray(d_syn, np.float64) - d_obs, kind, dt)
    return 2.0 * TRACE_TOL * np.linalg.norm(Wd) / np.linalg.norm(Wr)


def report(name, err, tol):
    print(f"[parity] {name}: rel err {err:.3e} (tol {tol:.1e})", flush=True)
    return err
