"""Iterative full-waveform inversion on top of the gradient path.

Section 2.1 inverts with limited-memory BFGS and section 3.1 with
preconditioned conjugate gradients, comparing three scalings of the gradient:
none, the shot illumination of eq. (1) (P = (4/v^6) H1) and the diagonal of
the localized subsurface-offset Hessian of section 3 (P = sum_h D(x, h)), each
applied as g / (P + eps max P).  The offset diagonal is taken with the
aperture-factor receiver model ("offset") or with the exact receiver term
from the receivers' impulse responses ("offset_exact", the conventional
misfit's diagonal, band up to `fmax` Hz).  This module provides both drivers
and a GPU objective that evaluates J, dJ/dv and the scaling through the HIP
library (fwi_misfit_value, fwi_gradient, fwi_offset_diag_exact,
fwi_precondition).

The drivers are plain host logic on NumPy arrays over any objective with

    value(v)       -> J
    value_grad(v)  -> (J, g, minv)   minv: the diagonal scaling 1/(P + eps max P)

so the same iteration can be run against another implementation of J.
Velocities stay inside [vmin, vmax] (projection after every step).

Line search: from a trial step that changes the model by at most `step0`
m/s, one more evaluation at the minimiser of the quadratic through J(0),
J'(0) and the trial value; the better of the two is taken, and the trial is
shrunk fourfold (at most four times) if neither decreases J.
"""
from __future__ import annotations

import time

import numpy as np


class GPUObjective:
    """J(v), dJ/dv and the diagonal scaling on the device, NumPy in and out."""

    def __init__(self, grid, geom, wavelet, d_obs, misfit="int", precond="shot", hmax=8, eps=1e-2,
                 rcv_model="pm", exec_=None, device="cuda", fmax=0.0, exact_runs=32):
        import torch
        from . import binding as B
        if precond not in ("none", "shot", "offset", "offset_exact"):
            raise ValueError(precond)
        self.B, self.torch = B, torch
        self.grid, self.geom = grid, B.GeometryC(geom)
        self.ntrace = geom.ntrace
        self.misfit, self.precond, self.hmax, self.eps, self.rcv = misfit, precond, hmax, eps, rcv_model
        self.exec, self.device = exec_, device
        self.wavelet, self.wstride = B._wavelet(wavelet, grid.nt_max, device)
        self.d_obs = B._dev(d_obs, torch.float32, device)
        self.ws_f = B.workspace(grid, self.geom, B.WS_FORWARD, exec_, device=device)
        self.ws_g = B.workspace(grid, self.geom, B.WS_GRADIENT, exec_, hmax if precond == "offset" else 0,
                                device=device)
        if precond == "offset_exact":
            self.fmax = fmax
            self.ex_x = B.make_exec(shots_in_flight=exact_runs)
            n = B.fwi_offset_diag_exact_workspace_bytes(grid, self.geom, self.ex_x, hmax, fmax, B.DFT_BF16X3)
            if n == 0:
                raise B.FwiError(B.FWI_ERR_ARG, B.last_error())
            self.ws_x = torch.empty(n, dtype=torch.uint8, device=device)
        self.evals = 0
        self.grads = 0

    def _v(self, v):
        return self.torch.as_tensor(np.asarray(v, np.float32), device=self.device).contiguous()

    def value(self, v) -> float:
        B, t = self.B, self.torch
        J = t.empty((), dtype=t.float64, device=self.device)
        B.fwi_misfit_value(self.grid, self.geom, self.exec, self._v(v), self.wavelet, self.wstride, self.d_obs,
                           self.misfit, J, self.ws_f, self.ws_f.numel())
        self.evals += 1
        return float(J)

    def value_grad(self, v):
        B, t, g_ = self.B, self.torch, self.grid
        vd = self._v(v)
        J = t.empty((), dtype=t.float64, device=self.device)
        grad = t.empty((g_.nz, g_.nx), dtype=t.float32, device=self.device)
        H1 = t.empty_like(grad) if self.precond == "shot" else None
        D = (t.empty((2 * self.hmax + 1, g_.nz, g_.nx), dtype=t.float32, device=self.device)
             if self.precond == "offset" else None)
        B.fwi_gradient(self.grid, self.geom, self.exec, vd, self.wavelet, self.wstride, self.d_obs, self.misfit,
                       J, grad, H1, self.hmax if D is not None else 0, self.rcv, D, self.ws_g, self.ws_g.numel())
        if self.precond == "offset_exact":
            D = t.empty((2 * self.hmax + 1, g_.nz, g_.nx), dtype=t.float32, device=self.device)
            B.fwi_offset_diag_exact(self.grid, self.geom, self.ex_x, vd, self.wavelet, self.wstride, self.hmax,
                                    self.fmax, B.DFT_BF16X3, D, self.ws_x, self.ws_x.numel())
        if self.precond == "none":
            minv = np.ones((g_.nz, g_.nx))
        else:
            ones = t.ones_like(grad)
            kind = B.PRECOND_SHOT if self.precond == "shot" else B.PRECOND_OFFSET
            hdiag = H1 if self.precond == "shot" else D
            minv = B.precondition(vd, ones, hdiag, g_, kind, self.hmax, self.eps,
                                  device=self.device).cpu().numpy().astype(np.float64)
        self.evals += 1
        self.grads += 1
        return float(J), grad.cpu().numpy().astype(np.float64), minv


def _project(v, vmin, vmax):
    return np.clip(v, vmin, vmax)


def line_search(obj, v, J0, g, d, step0, vmin, vmax):
    """Step along d (see the module notes).  Returns (alpha, J, v_new) with
    alpha = 0 when no decrease was found."""
    slope = float(np.sum(g * d))
    dmax = float(np.max(np.abs(d)))
    if not (slope < 0.0) or dmax == 0.0:
        return 0.0, J0, v
    a0 = step0 / dmax
    for _ in range(4):
        v1 = _project(v + a0 * d, vmin, vmax)
        J1 = obj.value(v1)
        curv = (J1 - J0 - slope * a0) / (a0 * a0)
        a = min(max(-slope / (2.0 * curv), 0.1 * a0), 10.0 * a0) if curv > 0.0 else 2.0 * a0
        v2 = _project(v + a * d, vmin, vmax)
        J2 = obj.value(v2)
        best = min((J1, a0, v1), (J2, a, v2), key=lambda c: c[0])
        if best[0] < J0:
            return best[1], best[0], best[2]
        a0 *= 0.25
    return 0.0, J0, v


def prcg(obj, v0, iters, step0=50.0, vmin=1400.0, vmax=4600.0, callback=None):
    """Preconditioned nonlinear conjugate gradients (Polak-Ribiere, restarted
    when beta < 0 or the direction is not a descent one)."""
    v = np.asarray(v0, np.float64).copy()
    J, g, minv = obj.value_grad(v)
    z = minv * g
    d = -z
    hist = [dict(iter=0, J=J, alpha=0.0, evals=obj.evals, t=time.perf_counter())]
    for k in range(1, iters + 1):
        alpha, Jn, vn = line_search(obj, v, J, g, d, step0, vmin, vmax)
        if alpha == 0.0:
            if np.array_equal(d, -z):
                break
            d = -z                       # restart on steepest descent
            alpha, Jn, vn = line_search(obj, v, J, g, d, step0, vmin, vmax)
            if alpha == 0.0:
                break
        v = vn
        Jn_, gn, minvn = obj.value_grad(v)
        zn = minvn * gn
        beta = max(0.0, float(np.sum(zn * (gn - g))) / float(np.sum(z * g)))
        d = -zn + beta * d
        if float(np.sum(gn * d)) >= 0.0:
            d = -zn
        J, g, z = Jn_, gn, zn
        hist.append(dict(iter=k, J=J, alpha=alpha, beta=beta, evals=obj.evals, t=time.perf_counter()))
        if callback:
            callback(k, v, hist[-1])
    return v, hist


def lbfgs(obj, v0, iters, m=5, step0=50.0, vmin=1400.0, vmax=4600.0, callback=None):
    """Limited-memory BFGS (two-loop recursion) with the diagonal scaling as
    the initial inverse Hessian, scaled by s.y / y.(M y) of the last pair."""
    v = np.asarray(v0, np.float64).copy()
    J, g, minv = obj.value_grad(v)
    S, Y = [], []
    hist = [dict(iter=0, J=J, alpha=0.0, evals=obj.evals, t=time.perf_counter())]
    for k in range(1, iters + 1):
        q = g.copy()
        rho = [1.0 / float(np.sum(y * s)) for s, y in zip(S, Y)]
        al = []
        for s, y, r in reversed(list(zip(S, Y, rho))):
            a = r * float(np.sum(s * q))
            al.append(a)
            q -= a * y
        gamma = float(np.sum(S[-1] * Y[-1])) / float(np.sum(Y[-1] * minv * Y[-1])) if S else 1.0
        r_ = gamma * minv * q
        for (s, y, r), a in zip(zip(S, Y, rho), reversed(al)):
            b = r * float(np.sum(y * r_))
            r_ += (a - b) * s
        d = -r_
        alpha, Jn, vn = line_search(obj, v, J, g, d, step0, vmin, vmax)
        if alpha == 0.0:
            S, Y = [], []
            d = -minv * g
            alpha, Jn, vn = line_search(obj, v, J, g, d, step0, vmin, vmax)
            if alpha == 0.0:
                break
        Jn_, gn, minvn = obj.value_grad(vn)
        s, y = vn - v, gn - g
        if float(np.sum(s * y)) > 1e-12 * float(np.sqrt(np.sum(s * s) * np.sum(y * y))):
            S.append(s)
            Y.append(y)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        v, J, g, minv = vn, Jn_, gn, minvn
        hist.append(dict(iter=k, J=J, alpha=alpha, evals=obj.evals, t=time.perf_counter()))
        if callback:
            callback(k, v, hist[-1])
    return v, hist


def main():
    """Convergence of the three scalings and the two misfits on the 256x96
    layered workload (the structure of the paper's two examples)."""
    import argparse
    import json
    from . import binding as B
    from .synthetic import layered_256x96
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--method", choices=["prcg", "lbfgs"], default="prcg")
    ap.add_argument("--misfits", default="l2,int")
    ap.add_argument("--preconds", default="none,shot,offset,offset_exact")
    args = ap.parse_args()
    w = layered_256x96()
    d_obs = B.forward(w.v_true, w.wavelet, w.grid, w.geom)
    err0 = float(np.linalg.norm(w.v_start - w.v_true))
    out = []
    for misfit in args.misfits.split(","):
        for pc in args.preconds.split(","):
            obj = GPUObjective(w.grid, w.geom, w.wavelet, d_obs, misfit, pc, hmax=w.hmax, fmax=4.0 * w.f_peak)
            t0 = time.perf_counter()
            run = prcg if args.method == "prcg" else lbfgs
            v, hist = run(obj, w.v_start, args.iters)
            rec = dict(misfit=misfit, precond=pc, method=args.method, iters=len(hist) - 1,
                       J_rel=[h["J"] / hist[0]["J"] for h in hist],
                       model_error_rel=float(np.linalg.norm(v - w.v_true)) / err0,
                       evaluations=obj.evals, gradients=obj.grads, seconds=time.perf_counter() - t0)
            print(json.dumps(rec), flush=True)
            out.append(rec)
    return out


if __name__ == "__main__":
    main()
