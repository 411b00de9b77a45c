"""FP64 oracle: Hessian diagonals and preconditioners.

TEST INFRASTRUCTURE ONLY (see ``oracle/acoustic.py``): no product code may
import it.

Follows section 1 (Gauss-Newton Hessian, the pseudo-diagonal of eq. (1), the
Plessix-Mulder aperture-weighted diagonal) and section 3 (Born operator
eq. (4), extended Born operator eq. (5), its adjoint eq. (6), and the
subsurface-offset Hessian, of which only the diagonal part is used).

Readings taken where the paper is silent or garbled:

* eq. (1) in the time domain: sum_omega omega^4 |u_s|^2 is, by Parseval,
  the energy of the second time derivative; its discrete form is
  E_s(x) = sum_m (D[m](x)/dt^2)^2 dt, H1 = sum_s E_s (no 4/v^6 factor, as
  printed in eq. (1)).
* the diagonal of the offset Hessian takes y = x and h_bar = h, with the
  receiver-side Green's functions replaced by the paper's own
  frequency-independent aperture factor (the Plessix-Mulder asinh term):
  D(x, h) = (4 / v(x)^6) sum_s E_s(x + h) A_s(x - h), h horizontal in cells,
  a term whose x+h or x-h leaves the model contributes 0.
* A_s(y) = asinh((X_max,s - y_x)/z_y) - asinh((X_min,s - y_x)/z_y), with
  X_min,s / X_max,s the extreme receiver x-positions (metres) of shot s and
  z_y = max((iz_y - iz_rec,s) h, h/2) measured from the shallowest receiver
  of the shot; ``rcv_model='none'`` uses A_s = 1 (the Shin form).
* the exact receiver term (``offset_diag_spectral``): the same diagonal with
  sum_r |G(x-h, r, omega)|^2 in place of the aperture factor, summed over the
  bins of L = 2 nt point DFTs of the discrete series (source side: D[j]/dt^2,
  j = 1 .. nt-1; receiver side: the impulse response of the scheme from the
  receiver, n = 0 .. nt-2, by reciprocity); with every bin it equals the
  extended-Born column norms over the whole response, not cut at the record's
  end.  A band limit fmax keeps the bins up to fmax.
* preconditioners: P_shot = (4/v^6) H1, P_off(x) = sum_h D(x, h),
  g_prec = g / (P + eps max P) with eps = 1e-2.
"""
from __future__ import annotations

import numpy as np

from .acoustic import Propagator, _source_term, forward, imaging, misfit, shot_gradient


def aperture_factor(grid, rec_iz, rec_ix, model="pm"):
    """A_s on the model grid [nz][nx] for one shot's receiver spread."""
    nz, nx, h = grid.nz, grid.nx, grid.dx
    if model in ("none", 1):
        return np.ones((nz, nx))
    rec_iz = np.asarray(rec_iz)
    rec_ix = np.asarray(rec_ix)
    xmin = float(rec_ix.min()) * h
    xmax = float(rec_ix.max()) * h
    iz_rec = int(rec_iz.min())
    z = np.maximum((np.arange(nz) - iz_rec) * h, 0.5 * h)[:, None]
    x = (np.arange(nx) * h)[None, :]
    return np.arcsinh((xmax - x) / z) - np.arcsinh((xmin - x) / z)


def offset_diag(v, E_list, A_list, hmax):
    """D[h + hmax][z][x] = (4/v^6) sum_s E_s(z, x+h) A_s(z, x-h)."""
    v = np.asarray(v, np.float64)
    nz, nx = v.shape
    D = np.zeros((2 * hmax + 1, nz, nx))
    for E, A in zip(E_list, A_list):
        for h in range(-hmax, hmax + 1):
            # x such that 0 <= x+h < nx and 0 <= x-h < nx
            lo, hi = abs(h), nx - abs(h)
            if lo >= hi:
                continue
            xs = np.arange(lo, hi)
            D[h + hmax][:, xs] += E[:, xs + h] * A[:, xs - h]
    return D * (4.0 / v ** 6)[None]


def shot_scaling(v, H1):
    """P_shot = (4/v^6) H1."""
    v = np.asarray(v, np.float64)
    return 4.0 / v ** 6 * H1


def offset_scaling(D):
    """P_off(x) = sum_h D(x, h)."""
    return np.sum(D, axis=0)


def precondition(g, P, eps=1e-2):
    """g / (P + eps * max P)."""
    P = np.asarray(P, np.float64)
    return np.asarray(g, np.float64) / (P + eps * P.max())


# --------------------------------------------------------------------------
# exact diagonals by explicit (extended) Born columns -- small grids only
# --------------------------------------------------------------------------
def extended_born_columns(v, grid, shot, wavelet, cells, kind="l2"):
    """Columns of the discretised extended Born operator (eq. (5)).

    For each (iz, ix, h) in ``cells`` the column is the recorded response
    to the model perturbation delta_v(x, h) = 1: the perturbation wavefield
    obeys the same scheme, started from zero, and in the update that yields
    du[m] it receives q(x-h) (2 / v(x)^3) D[m](x+h) at cell x-h, where
    D[m] = u[m] - 2u[m-1] + u[m-2] of the background wavefield u.  The source
    side is read at x+h, the receiver side enters at x-h and 2/v^3 is taken at
    the centre, as in eq. (5).  Returns [ncol, nrec, nt]; with kind='int' the
    time-integral weighting of eq. (2) (dt * running sum) is applied."""
    siz, six, riz, rix, nt = shot
    N = grid.nsponge
    v = np.asarray(v, np.float64)
    hist = []
    forward(v, grid, shot, wavelet, keep=hist)          # hist[n+1] = u[n]
    prop = Propagator(v, grid)
    ncol = len(cells)
    Z, X = prop.q.shape
    rz, rx = prop.cell(np.asarray(riz), np.asarray(rix))
    col = np.arange(ncol)
    inj_z = np.array([c[0] + N for c in cells])
    inj_x = np.array([c[1] - c[2] + N for c in cells])          # x - h
    src_x = np.array([c[1] + c[2] + N for c in cells])          # x + h
    for (iz, ix, h) in cells:
        assert 0 <= ix - h < grid.nx and 0 <= ix + h < grid.nx and 0 <= iz < grid.nz
    cen_v = np.array([v[c[0], c[1]] for c in cells])
    # step() adds dt^2 q (L du + extra): extra = (2/v^3) D / dt^2 gives q (2/v^3) D
    coef = 2.0 / cen_v ** 3 / (grid.dt ** 2)
    du_prev = np.zeros((ncol, Z, X))
    du = np.zeros((ncol, Z, X))
    out = np.zeros((ncol, len(riz), nt))
    for n in range(nt - 1):
        m = n + 1
        Dm = hist[m + 1] - 2.0 * hist[m] + hist[m - 1]          # D[m]
        extra = np.zeros((ncol, Z, X))
        extra[col, inj_z, inj_x] = coef * Dm[inj_z, src_x]
        dun = prop.step(du, du_prev, extra)
        du_prev, du = du, dun
        out[:, :, m] = du[:, rz, rx]
    if kind in ("int", 1):
        out = grid.dt * np.cumsum(out, axis=-1)
    return out


def offset_diag_exact(v, grid, geom, wavelet, cells, kind="l2"):
    """D_exact(x, h) = sum over shots, receivers, samples of the squared
    extended-Born column entries; at h = 0 this is diag(J^T J) of the
    Gauss-Newton Hessian.  ``cells`` is a list of (iz, ix, h)."""
    total = np.zeros(len(cells))
    for s in range(geom.nshot):
        shot = geom.shot(s)
        w = wavelet[s] if np.ndim(wavelet) == 2 else wavelet
        cols = extended_born_columns(v, grid, shot, np.asarray(w, np.float64), cells, kind)
        total += np.sum(cols * cols, axis=(1, 2))
    return total


def extended_image(v, grid, geom, wavelet, d_obs, kind, hmax, shots=None):
    """Offset-extended image: the gradient of J with respect to the extended
    model of eq. (5), i.e. the extended imaging condition of eq. (6) applied to
    the adjoint-state wavefields,

        I(x, h) = (2 / v(x)^3) sum_s sum_m lam_s[m](x - h) D_s[m](x + h),

    for horizontal offsets h = -hmax .. hmax (the receiver-side wavefield at
    x - h, the source side at x + h, 2/v^3 at the centre); terms with x - h or
    x + h outside the model vanish.  The h = 0 slice is the gradient g.
    Returns (J, I[2 hmax + 1][nz][nx])."""
    v = np.asarray(v, np.float64)
    nz, nx = v.shape
    shots = range(geom.nshot) if shots is None else shots
    acc = np.zeros((2 * hmax + 1, nz, nx))

    def visit(m, lam, D):
        for h in range(-hmax, hmax + 1):
            lo, hi = abs(h), nx - abs(h)
            if lo < hi:
                acc[h + hmax][:, lo:hi] += lam[:, lo - h:hi - h] * D[:, lo + h:hi + h]

    J = 0.0
    for s in shots:
        a, b = int(geom.rec_ptr[s]), int(geom.rec_ptr[s + 1])
        w = wavelet[s] if np.ndim(wavelet) == 2 else wavelet
        Js, _, _ = shot_gradient(v, grid, geom.shot(s), np.asarray(w, np.float64),
                                 np.asarray(d_obs[a:b], np.float64), kind, visit=visit)
        J += Js
    return J, acc * (2.0 / v ** 3)[None]


def born_shot(v, grid, shot, wavelet, dv):
    """Linearised traces dd = J dv of one shot: the Born operator of eq. (4)
    in the discrete scheme.  The perturbation wavefield obeys the scheme
    linearised in v at the model cells (padding frozen), started from zero;
    in the update that yields du[m] it receives dt^2 dq (L u[m-1] + s[m-1])
    with dq = 2 v dv, which inside the model equals (2 dv / v) D[m],
    D[m] = u[m] - 2u[m-1] + u[m-2].  Returns [nrec, nt]."""
    siz, six, riz, rix, nt = shot
    wavelet = np.asarray(wavelet, np.float64)
    v = np.asarray(v, np.float64)
    N, nz, nx = grid.nsponge, grid.nz, grid.nx
    prop = Propagator(v, grid)
    sz, sx = prop.cell(siz, six)
    rz, rx = prop.cell(np.asarray(riz), np.asarray(rix))
    # step() adds dt^2 q extra: extra = (2 dv / v^3) D / dt^2 gives (2 dv / v) D
    coef = np.zeros(prop.q.shape)
    coef[N:N + nz, N:N + nx] = 2.0 * np.asarray(dv, np.float64) / v ** 3 / grid.dt ** 2
    u_prev = np.zeros(prop.q.shape)
    u = np.zeros(prop.q.shape)
    du_prev = np.zeros(prop.q.shape)
    du = np.zeros(prop.q.shape)
    out = np.zeros((len(riz), nt))
    for n in range(nt - 1):
        un = prop.step(u, u_prev, _source_term(prop, prop.q.shape, np.float64, sz, sx, wavelet[n]))
        dun = prop.step(du, du_prev, coef * (un - 2.0 * u + u_prev))
        u_prev, u = u, un
        du_prev, du = du, dun
        out[:, n + 1] = du[rz, rx]
    return out


def born(v, grid, geom, wavelet, dv, shots=None):
    """Born data J dv [ntrace][nt_max] (zero past each shot's record)."""
    shots = range(geom.nshot) if shots is None else shots
    out = np.zeros((geom.ntrace, grid.nt_max))
    for s in shots:
        a, b = int(geom.rec_ptr[s]), int(geom.rec_ptr[s + 1])
        w = wavelet[s] if np.ndim(wavelet) == 2 else wavelet
        shot = geom.shot(s)
        out[a:b, :shot[4]] = born_shot(v, grid, shot, w, dv)
    return out


def gn_hvp(v, grid, geom, wavelet, dv, kind, shots=None):
    """Gauss-Newton Hessian times a model perturbation (section 1, H = J^T J
    with the data weighting of the misfit): returns
    (1/2 |W J dv|^2, J^T W^T W J dv) on the model cells, W = I (conventional)
    or the time integral of eq. (2).  The product is the gradient machinery
    with the Born data as the residual."""
    v = np.asarray(v, np.float64)
    shots = range(geom.nshot) if shots is None else shots
    Jb = 0.0
    G = np.zeros_like(v)
    for s in shots:
        shot = geom.shot(s)
        w = np.asarray(wavelet[s] if np.ndim(wavelet) == 2 else wavelet, np.float64)
        dd = born_shot(v, grid, shot, w, dv)
        Js, psi = misfit(dd, np.zeros_like(dd), kind, grid.dt)
        K = max(1, int(np.ceil(np.sqrt(shot[4]))))
        _, saves = forward(v, grid, shot, w, save_every=K)
        Gs, _ = imaging(v, grid, shot, w, psi, saves, K)
        Jb += Js
        G += Gs
    return Jb, 2.0 / v ** 3 * G


# --------------------------------------------------------------------------
# the offset diagonal with the exact receiver term (frequency domain)
# --------------------------------------------------------------------------
def spectral_bins(nt, dt, fmax=None):
    """DFT length L = 2 nt and the bins k = 0 .. K-1 kept, with their one-sided
    weights: a real series of L samples has sum_t x^2 = (1/L) sum_k m_k |X_k|^2,
    m_0 = m_{L/2} = 1, m_k = 2 in between.  fmax (Hz) keeps the bins with
    k / (L dt) <= fmax; None keeps all of them (the identity is then exact)."""
    L = 2 * int(nt)
    K = L // 2 + 1
    if fmax is not None:
        K = min(K, int(np.floor(fmax * L * dt + 1e-9)) + 1)
    m = np.full(K, 2.0)
    m[0] = 1.0
    if K == L // 2 + 1:
        m[-1] = 1.0
    return L, K, m


def green_series(v, grid, iz, ix, nt):
    """B(n, y) = h^2 u[n+1](y) on the model cells, n = 0 .. nt-2: the wavefield
    of a unit source term injected at (iz, ix) in the first update (a forward
    run with the wavelet [1, 0, 0, ...], which enters as 1/h^2).  The scheme is
    symmetric (a diagonal time operator plus the symmetric Laplacian), so
    B(n, y) is also the response at (iz, ix) n updates after a unit source
    term at y: the receiver-side Green's function of a receiver there."""
    N, nz, nx = grid.nsponge, grid.nz, grid.nx
    imp = np.zeros(nt)
    imp[0] = 1.0
    hist = []
    none = np.zeros(0, np.int64)
    forward(v, grid, (iz, ix, none, none, nt), imp, keep=hist)     # hist[n+1] = u[n]
    return np.array(hist[2:])[:, N:N + nz, N:N + nx] * grid.dx ** 2  # u[1] .. u[nt-1]


def source_series(v, grid, shot, wavelet):
    """A(i, y) = D[i+1](y) / dt^2 on the model cells, i = 0 .. nt-2, with
    D[j] = u[j] - 2u[j-1] + u[j-2]: the series the extended Born operator of
    eq. (5) injects (times 2/v^3)."""
    N, nz, nx = grid.nsponge, grid.nz, grid.nx
    hist = []
    forward(v, grid, shot, wavelet, keep=hist)
    u = np.array(hist)[:, N:N + nz, N:N + nx]                        # u[-1] .. u[nt-1]
    return (u[2:] - 2.0 * u[1:-1] + u[:-2]) / grid.dt ** 2


def power(series, L, K):
    """|X_k|^2, k = 0 .. K-1, of the L-point DFT along axis 0 (zero padded)."""
    X = np.fft.rfft(series, n=L, axis=0)[:K]
    return X.real ** 2 + X.imag ** 2


def offset_diag_spectral_cells(v, grid, geom, wavelet, cells, fmax=None, shots=None):
    """``offset_diag_spectral`` at the given cells only: D(x, h) for each
    (iz, ix, h) of ``cells`` (model indices, x - h and x + h inside the
    model), from the same series recorded at x + h (the shot's wavefield,
    ``source_series``) and at x - h (each receiver's unit-impulse wavefield,
    ``green_series``) instead of kept on the whole grid, so that a full-size
    grid fits in memory.  Returns an array of len(cells)."""
    v = np.asarray(v, np.float64)
    cz = np.array([c[0] for c in cells], np.int64)
    cx = np.array([c[1] for c in cells], np.int64)
    ch = np.array([c[2] for c in cells], np.int64)
    assert np.all(cx - np.abs(ch) >= 0) and np.all(cx + np.abs(ch) < v.shape[1])
    shots = range(geom.nshot) if shots is None else shots
    out = np.zeros(len(cells))
    for s in shots:
        shot = geom.shot(s)
        riz, rix, nt = shot[2], shot[3], int(shot[4])
        L, K, m = spectral_bins(nt, grid.dt, fmax)
        w = np.asarray(wavelet[s] if np.ndim(wavelet) == 2 else wavelet, np.float64)
        # source side: u[n] at x + h, n = 0 .. nt-1, behind u[-1] = 0
        u = forward(v, grid, (shot[0], shot[1], cz, cx + ch, nt), w)
        up = np.concatenate([np.zeros((len(cells), 1)), u], axis=1)
        A = (up[:, 2:] - 2.0 * up[:, 1:-1] + up[:, :-2]) / grid.dt ** 2
        PA = power(A.T, L, K)
        PB = np.zeros_like(PA)
        imp = np.zeros(nt)
        imp[0] = 1.0
        for r in range(len(riz)):
            # receiver side: h^2 u[n+1] at x - h of a unit source term at the receiver
            ur = forward(v, grid, (int(riz[r]), int(rix[r]), cz, cx - ch, nt), imp)
            PB += power((ur[:, 1:] * grid.dx ** 2).T, L, K)
        out += np.einsum("k,kc,kc->c", m, PA, PB) / L
    return out * 4.0 / v[cz, cx] ** 6


def offset_diag_spectral(v, grid, geom, wavelet, hmax, fmax=None, shots=None):
    """Diagonal of the subsurface-offset Hessian (section 3, y = x and
    h_bar = h) with the exact receiver term in place of the aperture factor:

        D(x, h) = (4 / v(x)^6) sum_s sum_{r in R_s} (1/L) sum_k m_k
                  |A_s_hat(x + h, k)|^2 |B_r_hat(x - h, k)|^2,

    the frequency-domain form of the paper's diagonal (source energy at x+h
    times the receiver Green's functions at x-h, frequency by frequency), on
    L = 2 nt point DFTs of the series ``source_series`` (A) and
    ``green_series`` (B), with the bins of ``spectral_bins``.  With every bin this is, by Parseval,
    sum_{s,r,t} c^2 over the extended-Born column of (x, h) convolved over the
    whole response (not cut at the record's end); for a record long enough to
    hold the response it is diag(J_ext^T J_ext) of the conventional misfit.
    Offsets are horizontal, zero where x+h or x-h leaves the model.  Returns
    D[2 hmax + 1][nz][nx]."""
    v = np.asarray(v, np.float64)
    nz, nx = v.shape
    shots = range(geom.nshot) if shots is None else shots
    D = np.zeros((2 * hmax + 1, nz, nx))
    green = {}
    for s in shots:
        shot = geom.shot(s)
        riz, rix, nt = shot[2], shot[3], int(shot[4])
        L, K, m = spectral_bins(nt, grid.dt, fmax)
        w = np.asarray(wavelet[s] if np.ndim(wavelet) == 2 else wavelet, np.float64)
        PA = power(source_series(v, grid, shot, w), L, K)
        PB = np.zeros_like(PA)
        for r in range(len(riz)):
            key = (int(riz[r]), int(rix[r]), nt, K)
            if key not in green:
                green[key] = power(green_series(v, grid, key[0], key[1], nt), L, K)
            PB += green[key]
        for h in range(-hmax, hmax + 1):
            lo, hi = abs(h), nx - abs(h)
            if lo >= hi:
                continue
            xs = np.arange(lo, hi)
            D[h + hmax][:, xs] += np.einsum("k,kzx,kzx->zx", m, PA[:, :, xs + h], PB[:, :, xs - h]) / L
    return D * (4.0 / v ** 6)[None]
