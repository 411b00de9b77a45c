"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in the oracle (on the CPU, through monkeypatch)
and checks that at least one of the pins in test_oracle_pins.py then fails.
Nothing here touches the HIP path.
"""
import numpy as np
import pytest

import oracle
import oracle.acoustic as ac
import oracle.hessian as hs
import test_oracle_pins as P
from paper_1406_1864_amd.synthetic import tiny_24x16


@pytest.fixture(scope="module")
def tiny():
    return tiny_24x16(nt=300)


def fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def plant(monkeypatch, module, name, value):
    """Replace `name` in its oracle module and in the package namespace."""
    monkeypatch.setattr(module, name, value)
    if hasattr(oracle, name):
        monkeypatch.setattr(oracle, name, value)


def test_wrong_stencil_weight_is_caught(monkeypatch):
    plant(monkeypatch, ac, "C8", (ac.C8[0], ac.C8[1], -ac.C8[2], ac.C8[3], ac.C8[4]))
    fails(P.test_laplacian_exact_on_polynomials)


def test_missing_source_scale_is_caught(monkeypatch):
    orig = ac._source_term

    def no_h2(prop, shape, dtype, siz, six, f):          # forgets the 1/h^2 of the point source
        return orig(prop, shape, dtype, siz, six, f) * prop.h * prop.h
    plant(monkeypatch, ac, "_source_term", no_h2)
    fails(P.test_hankel_analytic_green_function)


def test_amplifying_sponge_is_caught(monkeypatch):
    orig = ac.sponge_gamma
    plant(monkeypatch, ac, "sponge_gamma", lambda g: -orig(g))
    fails(P.test_sponge_absorbs)


def test_doubled_sponge_damping_is_caught(monkeypatch):
    orig = ac.sponge_gamma
    plant(monkeypatch, ac, "sponge_gamma", lambda g: 2.0 * orig(g))
    fails(P.test_sponge_normal_incidence_reflection)


def test_halved_sponge_damping_is_caught(monkeypatch):
    orig = ac.sponge_gamma
    plant(monkeypatch, ac, "sponge_gamma", lambda g: 0.5 * orig(g))
    fails(P.test_sponge_normal_incidence_reflection)


def test_offset_scaling_mean_is_caught(monkeypatch):
    plant(monkeypatch, hs, "offset_scaling", lambda D: np.mean(D, axis=0))
    fails(P.test_offset_scaling_sums_every_offset)


def test_offset_scaling_zero_offset_only_is_caught(monkeypatch):
    plant(monkeypatch, hs, "offset_scaling", lambda D: np.asarray(D)[np.asarray(D).shape[0] // 2])
    fails(P.test_offset_scaling_sums_every_offset)


def test_exclusive_time_integral_is_caught(monkeypatch):
    def exclusive(d_syn, d_obs, dt):
        r = np.asarray(d_syn, np.float64) - np.asarray(d_obs, np.float64)
        R = dt * (np.cumsum(r, axis=-1) - r)
        J = 0.5 * float(np.sum(R * R))
        return J, dt * np.cumsum(R[..., ::-1], axis=-1)[..., ::-1]
    plant(monkeypatch, ac, "misfit_time_integral", exclusive)
    fails(P.test_time_integral_adjoint_source_explicit_matrix)


def test_adjoint_source_scale_is_caught(monkeypatch, tiny):
    orig = ac.adjoint

    def scaled(v, grid, shot, psi):                       # injects dt^2 q psi instead of q psi
        return orig(v, grid, shot, np.asarray(psi) * grid.dt ** 2)
    plant(monkeypatch, ac, "adjoint", scaled)
    fails(P.test_dot_product_adjoint, tiny)


def test_missing_gradient_factor_is_caught(monkeypatch, tiny):
    orig = ac.gradient

    def one_over_v3(v, grid, geom, wavelet, d_obs, kind, shots=None, return_parts=False):
        out = orig(v, grid, geom, wavelet, d_obs, kind, shots, return_parts)
        return (out[0], out[1] / 2.0) + tuple(out[2:])   # drops the 2 of 2/v^3
    plant(monkeypatch, ac, "gradient", one_over_v3)
    fails(P.test_gradient_equals_jacobian_transpose_residual, tiny, P.complex_step_jacobian(tiny, P.SAMPLE_CELLS), "int")


def test_shifted_second_difference_is_caught(monkeypatch, tiny):
    """Correlating lam[m] with D[m+1] instead of D[m]."""
    def shifted(v, grid, shot, wavelet, d_obs, kind, K=None):
        siz, six, riz, rix, nt = shot
        N, nz, nx = grid.nsponge, grid.nz, grid.nx
        hist = []
        traces = ac.forward(v, grid, shot, wavelet, keep=hist)
        J, psi = ac.misfit(traces, d_obs[..., :nt], kind, grid.dt)
        G = np.zeros((nz, nx))
        E = np.zeros((nz, nx))
        sl = (slice(N, N + nz), slice(N, N + nx))
        for m, lam in ac.adjoint(v, grid, shot, psi):
            mm = min(m + 1, nt - 1)
            D = (hist[mm + 1] - 2 * hist[mm] + hist[mm - 1])[sl]
            G += lam[sl] * D
            E += D * D / grid.dt ** 3
        return J, G, E
    plant(monkeypatch, ac, "shot_gradient", shifted)
    fails(P.test_gradient_equals_jacobian_transpose_residual, tiny, P.complex_step_jacobian(tiny, P.SAMPLE_CELLS), "l2")


def test_missing_illumination_dt_is_caught(monkeypatch, tiny):
    orig = ac.illumination
    plant(monkeypatch, ac, "illumination", lambda *a, **k: [E * a[1].dt for E in orig(*a, **k)])
    fails(P.test_illumination_parseval, tiny)


def test_swapped_aperture_ends_are_caught(monkeypatch):
    orig = hs.aperture_factor

    def swapped(grid, rec_iz, rec_ix, model="pm"):
        return -orig(grid, rec_iz, rec_ix, model)
    plant(monkeypatch, hs, "aperture_factor", swapped)
    fails(P.test_aperture_factor_is_inverse_distance_integral)


def test_swapped_offset_sides_are_caught(monkeypatch):
    def swapped(v, E_list, A_list, hmax):
        v = np.asarray(v, np.float64)
        nz, nx = v.shape
        D = np.zeros((2 * hmax + 1, nz, nx))
        for E, A in zip(E_list, A_list):
            for h in range(-hmax, hmax + 1):
                lo, hi = abs(h), nx - abs(h)
                xs = np.arange(lo, hi)
                D[h + hmax][:, xs] += E[:, xs - h] * A[:, xs + h]   # source side at x-h
        return D * (4.0 / v ** 6)[None]
    plant(monkeypatch, hs, "offset_diag", swapped)
    fails(P.test_offset_diagonal_special_cases)


def test_extended_born_side_swap_is_caught(monkeypatch, tiny):
    orig = hs.extended_born_columns

    def swapped(v, grid, shot, wavelet, cells, kind="l2"):
        return orig(v, grid, shot, wavelet, [(iz, ix, -h) for (iz, ix, h) in cells], kind)
    plant(monkeypatch, hs, "extended_born_columns", swapped)
    fails(P.test_extended_born_column_is_a_point_source_response, tiny)


def test_extended_image_side_swap_is_caught(monkeypatch, tiny):
    """Receiver side read at x+h and source side at x-h."""
    def swapped(v, grid, geom, wavelet, d_obs, kind, hmax, shots=None):
        v = np.asarray(v, np.float64)
        nz, nx = v.shape
        acc = np.zeros((2 * hmax + 1, nz, nx))

        def visit(m, lam, D):
            for h in range(-hmax, hmax + 1):
                lo, hi = abs(h), nx - abs(h)
                acc[h + hmax][:, lo:hi] += lam[:, lo + h:hi + h] * D[:, lo - h:hi - h]
        J = 0.0
        for s in range(geom.nshot):
            a, b = int(geom.rec_ptr[s]), int(geom.rec_ptr[s + 1])
            Js, _, _ = ac.shot_gradient(v, grid, geom.shot(s), np.asarray(wavelet, np.float64),
                                        np.asarray(d_obs[a:b], np.float64), kind, visit=visit)
            J += Js
        return J, acc * (2.0 / v ** 3)[None]
    plant(monkeypatch, hs, "extended_image", swapped)
    fails(P.test_extended_image_is_extended_born_adjoint, tiny, "l2")


def test_born_missing_factor_is_caught(monkeypatch, tiny):
    """Born source (dv / v) D instead of (2 dv / v) D."""
    orig = hs.born_shot

    def half(v, grid, shot, wavelet, dv):
        return orig(v, grid, shot, wavelet, 0.5 * np.asarray(dv))
    plant(monkeypatch, hs, "born_shot", half)
    fails(P.test_born_is_the_complex_step_derivative, tiny)


def test_eq3_unshifted_pairing_is_caught(monkeypatch, tiny):
    """u[m] paired with lam[m] instead of u[m-1] with lam[m]."""
    def unshifted(v, grid, geom, wavelet, d_obs, shots=None):
        v = np.asarray(v, np.float64)
        N, nz, nx = grid.nsponge, grid.nz, grid.nx
        J, G = 0.0, np.zeros_like(v)
        for s in range(geom.nshot):
            a, b = int(geom.rec_ptr[s]), int(geom.rec_ptr[s + 1])
            shot = geom.shot(s)
            hist = []
            traces = ac.forward(v, grid, shot, np.asarray(wavelet, np.float64), keep=hist)
            J += ac.misfit_time_integral(traces, d_obs[a:b, :shot[4]], grid.dt)[0]
            r = traces - d_obs[a:b, :shot[4]]
            for m, lam in ac.adjoint(v, grid, shot, r):
                G += hist[m + 1][N:N + nz, N:N + nx] * lam[N:N + nz, N:N + nx]
        return J, -(2.0 / v ** 3) * grid.dt ** 2 * G
    plant(monkeypatch, ac, "gradient_eq3_literal", unshifted)
    fails(P.test_eq3_literal_plus_end_of_record_term_is_the_exact_gradient, tiny)


def test_free_surface_mirror_sign_is_caught(monkeypatch):
    """Even (rigid) image instead of the odd (pressure-free) one."""
    def even(self, u):
        N = self.N
        g = u.copy()
        g[..., :N, :] = 0.0
        for k in range(1, 4):
            g[..., N - 1 - k, :] = u[..., N - 1 + k, :]
        return g
    monkeypatch.setattr(ac.Propagator, "mirror", even)
    fails(P.test_free_surface_is_the_antisymmetric_image)


def test_two_sided_bin_weights_dropped_are_caught(monkeypatch):
    """Every bin weighted 1 (the negative frequencies forgotten)."""
    orig = hs.spectral_bins

    def flat(nt, dt, fmax=None):
        L, K, m = orig(nt, dt, fmax)
        return L, K, np.ones_like(m)
    plant(monkeypatch, hs, "spectral_bins", flat)
    fails(P.test_spectral_bins_are_parseval)
    fails(P.test_offset_diag_spectral_is_full_response_column_norm)


def test_green_series_one_step_early_is_caught(monkeypatch):
    """u[n] instead of u[n+1] for the receiver impulse response."""
    def early(v, grid, iz, ix, nt):
        N, nz, nx = grid.nsponge, grid.nz, grid.nx
        imp = np.zeros(nt)
        imp[0] = 1.0
        hist = []
        none = np.zeros(0, np.int64)
        ac.forward(v, grid, (iz, ix, none, none, nt), imp, keep=hist)
        return np.array(hist[1:-1])[:, N:N + nz, N:N + nx] * grid.dx ** 2
    plant(monkeypatch, hs, "green_series", early)
    fails(P.test_extended_born_column_is_receiver_impulse_convolution)


def test_spectral_offset_sides_swapped_are_caught(monkeypatch):
    """Source side read at x-h, receiver side at x+h."""
    orig = hs.offset_diag_spectral

    def swapped(v, grid, geom, wavelet, hmax, fmax=None, shots=None):
        D = orig(v, grid, geom, wavelet, hmax, fmax, shots)
        return D[::-1].copy()  # D(x, -h)
    plant(monkeypatch, hs, "offset_diag_spectral", swapped)
    fails(P.test_offset_diag_spectral_is_full_response_column_norm)
