"""FP64 CPU oracle: acoustic propagation, misfits, adjoint-state gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It is deliberately plain and
slow: NumPy in float64 (or complex128 for complex-step checks), the steps of
the method in the paper's order, no blocking and no fusion.  It shares no
code with the HIP path.

What it follows (Huang, Wang & Ren, "Two new gradient precondition schemes
for full waveform inversion"):

* section 2: the data-weighted least-squares misfit J(v) over shots,
  receivers and time, with the constant-density acoustic equation as the
  forward model; W_d = I is the conventional misfit;
* section 2, the conventional gradient: zero-lag cross-correlation of the
  second time derivative of the forward wavefield with the back-propagated
  residual wavefield, scaled by 2/v^3;
* eq. (2): the time-integral misfit, W_d u = integral_0^t u;
* eq. (3): its gradient by the adjoint-state method.  The oracle computes the
  *exact discrete* gradient of eq. (2) (the adjoint of the scheme below with
  the time-integral weighting folded into the adjoint source), not the
  continuous eq. (3) formula, which drops an end-of-record term.

The paper names only "time domain finite difference" and gives no order,
boundary or source model.  The discrete readings used here are:

* Laplacian: 8th-order central, 17 points, weights
  (-205/72, 8/5, -1/5, 8/315, -1/560) / h^2, zero outside the padded grid;
* scheme: (1+g) u[n+1] = 2 u[n] - (1-g) u[n-1] + dt^2 q (L u[n] + s[n]),
  q = v_pad^2, u[0] = u[-1] = 0, n = 0 .. nt-2;
* sponge: N cells padded outside the model on all four sides by edge
  replication of v; g = (dt/2) eta_max (d/N)^2 with d the max-norm cell
  distance into the sponge and eta_max = 3 v_ref ln(1000) / (2 N h);
* optional free surface (``grid.free_surface``): no sponge above the model;
  u = 0 on the padded row just above the model and the three rows above
  that hold -u of the mirrored model rows (antisymmetric image about that
  row), so the Laplacian stays symmetric and the adjoint keeps its form;
* source s[n] = f[n] / h^2 at one cell; receivers record u[n] at cells,
  n = 0 .. nt-1;
* misfits: J_L2 = 1/2 sum r^2 and J_int = 1/2 sum R^2 with
  R[n] = dt sum_{k<=n} r[k], r = d_syn - d_obs;
* adjoint: (1+g) lam[m] = 2 lam[m+1] - (1-g) lam[m+2] + dt^2 q L lam[m+1]
  + q sum_r psi_r[m] e_r, m = nt-1 .. 1, lam[nt] = lam[nt+1] = 0, with
  psi = dJ/d(u at receivers);
* gradient on model cells (padding frozen):
  g(x) = (2/v^3) sum_{m=1}^{nt-1} lam[m](x) D[m](x),
  D[m] = u[m] - 2 u[m-1] + u[m-2];
* eq. (1), time-domain Parseval form:
  E_s(x) = sum_m (D[m](x)/dt^2)^2 dt, H1 = sum_s E_s.
"""
from __future__ import annotations

import math

import numpy as np

# 8th-order second-derivative weights (c0 applies to the centre of one axis)
C8 = (-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0)

# stability bound of the scheme: v dt / h <= 2 / sqrt(2 * sum |c| weights)
CFL_LIMIT = 2.0 / math.sqrt(2.0 * (abs(C8[0]) + 2.0 * sum(abs(c) for c in C8[1:])))


def laplacian(u, h):
    """8th-order 17-point Laplacian over the last two axes, zero outside."""
    out = (2.0 * C8[0]) * u
    for k in range(1, 5):
        c = C8[k]
        out[..., k:, :] += c * u[..., :-k, :]
        out[..., :-k, :] += c * u[..., k:, :]
        out[..., :, k:] += c * u[..., :, :-k]
        out[..., :, :-k] += c * u[..., :, k:]
    return out / (h * h)


def sponge_gamma(grid):
    """Damping factor g(z, x) = (dt/2) eta_max (d/N)^2 on the padded grid."""
    N, nz, nx = grid.nsponge, grid.nz, grid.nx
    iz = np.arange(nz + 2 * N)
    ix = np.arange(nx + 2 * N)
    dz = np.maximum(np.maximum(N - iz, iz - (N + nz - 1)), 0)
    dx = np.maximum(np.maximum(N - ix, ix - (N + nx - 1)), 0)
    d = np.maximum(dz[:, None], dx[None, :]).astype(np.float64)
    eta_max = 3.0 * grid.v_ref * math.log(1e3) / (2.0 * N * grid.dx) if N > 0 else 0.0
    return 0.5 * grid.dt * eta_max * (d / max(N, 1)) ** 2


def padded_q(v, N):
    """q = v_pad^2, with v edge-replicated into the sponge (last two axes)."""
    v = np.asarray(v)
    pad = [(0, 0)] * (v.ndim - 2) + [(N, N), (N, N)]
    vp = np.pad(v, pad, mode="edge")
    return vp * vp


class Propagator:
    """One medium on the padded grid; ``step`` is the damped leapfrog update."""

    def __init__(self, v, grid):
        self.grid = grid
        self.N = grid.nsponge
        dt = grid.dt
        v = np.asarray(v)
        if not np.iscomplexobj(v):
            v = v.astype(np.float64)
        self.v = v
        self.q = padded_q(v, self.N)
        g = sponge_gamma(grid)
        self.a_plus = 1.0 + g
        self.a_minus = 1.0 - g
        self.dt2q = dt * dt * self.q
        self.h = grid.dx
        self.fs = bool(getattr(grid, "free_surface", False))

    def mirror(self, u):
        """Free surface: rows above the model replaced by the antisymmetric
        image about padded row N-1 (which is zero)."""
        N = self.N
        g = u.copy()
        g[..., :N, :] = 0.0
        for k in range(1, 4):
            g[..., N - 1 - k, :] = -u[..., N - 1 + k, :]
        return g

    def step(self, u, u_prev, extra):
        """Return u[n+1] from u[n], u[n-1]; ``extra`` is added to L u[n]."""
        if self.fs:
            u = self.mirror(u)
        rhs = 2.0 * u - self.a_minus * u_prev + self.dt2q * (laplacian(u, self.h) + extra)
        out = rhs / self.a_plus
        if self.fs:
            out[..., :self.N, :] = 0.0           # above the surface: not part of the medium
        return out

    def cell(self, iz, ix):
        return iz + self.N, ix + self.N


def _source_term(prop, shape, dtype, siz, six, f):
    s = np.zeros(shape, dtype)
    s[..., siz, six] = np.float64(f) / (prop.h * prop.h)
    return s


def forward(v, grid, shot, wavelet, keep=None, save_every=None):
    """Forward-model one shot.

    ``shot`` = (src_iz, src_ix, rec_iz[], rec_ix[], nt).  Returns the traces
    ``[..., nrec, nt]`` (receiver samples u[n], n = 0 .. nt-1) and, on request,
    ``keep``: a list with u[n] for every n (n = -1 .. nt-1) or ``save_every``:
    a dict {n: (u[n-1], u[n])} at n = 0, K, 2K, ...
    """
    siz, six, riz, rix, nt = shot
    wavelet = np.asarray(wavelet, np.float64)
    prop = Propagator(v, grid)
    Z, X = prop.q.shape[-2:]
    dtype = np.result_type(prop.q.dtype, np.float64)
    shape = prop.q.shape
    u_prev = np.zeros(shape, dtype)          # u[-1]
    u = np.zeros(shape, dtype)               # u[0]
    sz, sx = prop.cell(siz, six)
    rz, rx = prop.cell(np.asarray(riz), np.asarray(rix))
    traces = np.zeros(shape[:-2] + (len(riz), nt), dtype)
    traces[..., 0] = u[..., rz, rx]
    hist = None
    if keep is not None:
        hist = [u_prev.copy(), u.copy()]
    saves = {}
    if save_every:
        saves[0] = (u_prev.copy(), u.copy())
    for n in range(nt - 1):
        src = _source_term(prop, shape, dtype, sz, sx, wavelet[n])
        u_next = prop.step(u, u_prev, src)
        u_prev, u = u, u_next
        traces[..., n + 1] = u[..., rz, rx]
        if hist is not None:
            hist.append(u.copy())
        if save_every and (n + 1) % save_every == 0:
            saves[n + 1] = (u_prev.copy(), u.copy())
    if keep is not None:
        keep.extend(hist)
    if save_every:
        return traces, saves
    return traces


# --------------------------------------------------------------------------
# misfits (section 2 and eq. (2))
# --------------------------------------------------------------------------
def misfit_l2(d_syn, d_obs):
    """Conventional misfit, W_d = I: J = 1/2 sum r^2, psi = r."""
    r = np.asarray(d_syn, np.float64) - np.asarray(d_obs, np.float64)
    return 0.5 * float(np.sum(r * r)), r


def misfit_time_integral(d_syn, d_obs, dt):
    """Eq. (2): J = 1/2 sum R^2 with R[n] = dt sum_{k<=n} r[k] (inclusive
    rectangle rule).  psi[n] = dJ/dr[n] = dt sum_{k>=n} R[k]."""
    r = np.asarray(d_syn, np.float64) - np.asarray(d_obs, np.float64)
    R = dt * np.cumsum(r, axis=-1)
    J = 0.5 * float(np.sum(R * R))
    psi = dt * np.cumsum(R[..., ::-1], axis=-1)[..., ::-1]
    return J, psi


def misfit(d_syn, d_obs, kind, dt):
    if kind in ("l2", 0):
        return misfit_l2(d_syn, d_obs)
    if kind in ("int", "time_integral", 1):
        return misfit_time_integral(d_syn, d_obs, dt)
    raise ValueError(kind)


# --------------------------------------------------------------------------
# adjoint and gradient
# --------------------------------------------------------------------------
def adjoint(v, grid, shot, psi):
    """Back-propagate psi ``[nrec, nt]``; yields (m, lam[m]) for m = nt-1 .. 1.

    The recursion is the exact transpose of ``forward``'s scheme, rescaled by
    q so that it has the same form as the forward update: the residual enters
    as q * psi at the receiver cells."""
    siz, six, riz, rix, nt = shot
    prop = Propagator(v, grid)
    shape = prop.q.shape
    dtype = np.result_type(prop.q.dtype, np.asarray(psi).dtype, np.float64)
    rz, rx = prop.cell(np.asarray(riz), np.asarray(rix))
    lam1 = np.zeros(shape, dtype)    # lam[m+1]
    lam2 = np.zeros(shape, dtype)    # lam[m+2]
    h2 = prop.h * prop.h
    for m in range(nt - 1, 0, -1):
        inj = np.zeros(shape, dtype)
        np.add.at(inj, (Ellipsis, rz, rx), psi[..., m])
        # step() adds dt^2 q (L lam + extra); q psi == dt^2 q (psi / dt^2)
        lam = prop.step(lam1, lam2, inj / (grid.dt * grid.dt))
        lam2, lam1 = lam1, lam
        yield m, lam


def source_adjoint(v, grid, shot, d):
    """Transpose of wavelet -> traces: returns (F^T d)[n], n = 0 .. nt-1,
    equal to (dt^2/h^2) lam[n+1](source cell) (zero for n = nt-1)."""
    siz, six, riz, rix, nt = shot
    prop = Propagator(v, grid)
    sz, sx = prop.cell(siz, six)
    out = np.zeros(np.asarray(d).shape[:-2] + (nt,), np.float64)
    fac = grid.dt * grid.dt / (grid.dx * grid.dx)
    for m, lam in adjoint(v, grid, shot, d):
        out[..., m - 1] = fac * lam[..., sz, sx]
    return out


def shot_gradient(v, grid, shot, wavelet, d_obs, kind, K=None, visit=None):
    """J_s, G_s = sum_m lam[m] D[m] and E_s = sum_m (D[m]/dt^2)^2 dt on the
    model grid, for one shot.  ``visit(m, lam[m], D[m])`` (model cells), if
    given, sees every pair that enters G_s."""
    siz, six, riz, rix, nt = shot
    wavelet = np.asarray(wavelet, np.float64)
    K = K or max(1, int(math.ceil(math.sqrt(nt))))
    traces, saves = forward(v, grid, shot, wavelet, save_every=K)
    J, psi = misfit(traces, d_obs[..., :nt], kind, grid.dt)
    G, E = imaging(v, grid, shot, wavelet, psi, saves, K, visit)
    return J, G, E


def imaging(v, grid, shot, wavelet, psi, saves, K, visit=None):
    """G_s = sum_m lam[m] D[m] and E_s = sum_m (D[m]/dt^2)^2 dt on the model
    grid, with lam back-propagated from the adjoint source ``psi`` [nrec, nt]
    and D[m] = u[m] - 2u[m-1] + u[m-2] of the source wavefield.

    Checkpointing (oracle's own, exact): ``saves`` holds (u[n-1], u[n]) every
    K steps in FP64 (``forward(..., save_every=K)``); each K-step segment is
    recomputed *forward* from its saved state and the adjoint runs through
    it."""
    siz, six, riz, rix, nt = shot
    wavelet = np.asarray(wavelet, np.float64)
    N, nz, nx = grid.nsponge, grid.nz, grid.nx
    prop = Propagator(v, grid)
    sz, sx = prop.cell(siz, six)
    G = np.zeros(prop.q.shape[:-2] + (nz, nx), np.result_type(prop.q.dtype, np.asarray(psi).dtype, np.float64))
    E = np.zeros((nz, nx), np.float64)
    interior = (Ellipsis, slice(N, N + nz), slice(N, N + nx))

    lam_iter = adjoint(v, grid, shot, psi)
    # segment j covers m in [jK+1, (j+1)K] and needs u[jK-1] .. u[(j+1)K]
    nseg = (nt - 1 + K - 1) // K
    pending = next(lam_iter, None)
    for j in range(nseg - 1, -1, -1):
        m_lo, m_hi = j * K + 1, min((j + 1) * K, nt - 1)
        up, uc = saves[j * K]
        seg = {j * K - 1: up, j * K: uc}
        for n in range(j * K, m_hi):
            src = _source_term(prop, prop.q.shape, uc.dtype, sz, sx, wavelet[n])
            un = prop.step(uc, up, src)
            up, uc = uc, un
            seg[n + 1] = uc
        for m in range(m_hi, m_lo - 1, -1):
            mm, lam = pending
            assert mm == m
            D = (seg[m] - 2.0 * seg[m - 1] + seg[m - 2])[interior]
            G += lam[interior] * D
            if visit is not None:
                visit(m, lam[interior], D)
            E += np.real(D * np.conj(D)) / grid.dt ** 3
            pending = next(lam_iter, None)
    return G, E


def gradient(v, grid, geom, wavelet, d_obs, kind, shots=None, return_parts=False):
    """Sum over shots: J, g = dJ/dv (model cells, padding frozen) and
    H1 = sum_s E_s (eq. (1), time-domain form).  ``wavelet`` is [nt_max] or
    [nshot][nt_max]; ``d_obs`` is [ntrace][nt_max]."""
    v = np.asarray(v, np.float64)
    shots = range(geom.nshot) if shots is None else shots
    J = 0.0
    G = np.zeros_like(v)
    H1 = np.zeros_like(v)
    E_list = []
    for s in shots:
        shot = geom.shot(s)
        a, b = int(geom.rec_ptr[s]), int(geom.rec_ptr[s + 1])
        w = wavelet[s] if np.ndim(wavelet) == 2 else wavelet
        Js, Gs, Es = shot_gradient(v, grid, shot, np.asarray(w, np.float64),
                                   np.asarray(d_obs[a:b], np.float64), kind)
        J += Js
        G += Gs
        H1 += Es
        E_list.append(Es)
    g = 2.0 / v ** 3 * G
    if return_parts:
        return J, g, H1, E_list
    return J, g, H1


def illumination(v, grid, geom, wavelet, shots=None):
    """E_s for each shot from the forward wavefield alone (eq. (1))."""
    N, nz, nx = grid.nsponge, grid.nz, grid.nx
    shots = range(geom.nshot) if shots is None else shots
    out = []
    for s in shots:
        siz, six, riz, rix, nt = geom.shot(s)
        w = np.asarray(wavelet[s] if np.ndim(wavelet) == 2 else wavelet, np.float64)
        prop = Propagator(v, grid)
        sz, sx = prop.cell(siz, six)
        u_prev = np.zeros(prop.q.shape)
        u = np.zeros(prop.q.shape)
        E = np.zeros((nz, nx))
        for n in range(nt - 1):
            src = _source_term(prop, prop.q.shape, np.float64, sz, sx, w[n])
            un = prop.step(u, u_prev, src)
            D = (un - 2.0 * u + u_prev)[N:N + nz, N:N + nx]
            E += D * D / grid.dt ** 3
            u_prev, u = u, un
        out.append(E)
    return out


def gradient_eq3_literal(v, grid, geom, wavelet, d_obs, shots=None):
    """Eq. (3) taken literally: the source wavefield u itself (not its second
    time derivative) correlated with the adjoint wavefield of the *plain*
    residual, in the discrete form whose difference from the exact eq. (2)
    gradient is a pure end-of-record term:

        g3(x) = -(2/v^3) dt^2 sum_s sum_n u_s[n](x) lam_r,s[n+1](x),

    lam_r the adjoint of ``adjoint`` driven by psi = r (W_d = I).  Summing the
    exact gradient by parts twice in time gives
        g_int = g3 + (2/v^3) sum_s sum_n u_s[n] eps_s[n],
    eps_s the adjoint driven only at n = nt-1 by dt R[nt-1] = dt^2 sum_n r[n]
    (the record does not end at rest), which ``end_of_record_term`` returns.
    Returns (J_int, g3)."""
    v = np.asarray(v, np.float64)
    shots = range(geom.nshot) if shots is None else shots
    nz, nx, N = grid.nz, grid.nx, grid.nsponge
    J = 0.0
    G = np.zeros_like(v)
    for s in shots:
        a, b = int(geom.rec_ptr[s]), int(geom.rec_ptr[s + 1])
        shot = geom.shot(s)
        nt = shot[4]
        w = np.asarray(wavelet[s] if np.ndim(wavelet) == 2 else wavelet, np.float64)
        hist = []
        traces = forward(v, grid, shot, w, keep=hist)          # hist[n + 1] = u[n]
        Js, _ = misfit_time_integral(traces, d_obs[a:b, :nt], grid.dt)
        _, r = misfit_l2(traces, d_obs[a:b, :nt])
        J += Js
        for m, lam in adjoint(v, grid, shot, r):
            G += hist[m][N:N + nz, N:N + nx] * lam[N:N + nz, N:N + nx]     # u[m-1] lam[m]
    return J, -(2.0 / v ** 3) * grid.dt ** 2 * G


def end_of_record_term(v, grid, geom, wavelet, d_obs, shots=None):
    """(2/v^3) sum_s sum_n u_s[n] eps_s[n]: the adjoint eps is driven only at
    the last sample, by dt R[nt-1] at each receiver (eq. (2) integral of the
    whole residual trace)."""
    v = np.asarray(v, np.float64)
    shots = range(geom.nshot) if shots is None else shots
    nz, nx, N = grid.nz, grid.nx, grid.nsponge
    G = np.zeros_like(v)
    for s in shots:
        a, b = int(geom.rec_ptr[s]), int(geom.rec_ptr[s + 1])
        shot = geom.shot(s)
        nt = shot[4]
        w = np.asarray(wavelet[s] if np.ndim(wavelet) == 2 else wavelet, np.float64)
        hist = []
        traces = forward(v, grid, shot, w, keep=hist)
        r = traces - np.asarray(d_obs[a:b, :nt], np.float64)
        src = np.zeros_like(r)
        src[:, nt - 1] = grid.dt * grid.dt * np.sum(r, axis=-1)
        for m, eps in adjoint(v, grid, shot, src):
            G += hist[m + 1][N:N + nz, N:N + nx] * eps[N:N + nz, N:N + nx]   # u[m] eps[m]
    return 2.0 / v ** 3 * G


def forward_traces(v, grid, geom, wavelet, shots=None):
    """Traces [ntrace][nt_max] of all (or the given) shots, zero past nt_s."""
    shots = list(range(geom.nshot)) if shots is None else list(shots)
    out = np.zeros((geom.ntrace, grid.nt_max))
    for s in shots:
        shot = geom.shot(s)
        w = wavelet[s] if np.ndim(wavelet) == 2 else wavelet
        a, b = int(geom.rec_ptr[s]), int(geom.rec_ptr[s + 1])
        out[a:b, :shot[4]] = forward(np.asarray(v, np.float64), grid, shot, np.asarray(w, np.float64))
    return out
