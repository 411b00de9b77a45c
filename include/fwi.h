/*
 * fwi.h -- C ABI of libfwi: the preconditioned FWI gradient hot path on MI355X.
 *
 * Method: Huang, Wang & Ren, "Two new gradient precondition schemes for full
 * waveform inversion".  The library computes, for a 2D constant-density
 * acoustic medium and many shots,
 *   - the forward wavefield and the recorded traces (section 2: d is recorded,
 *     u is synthesised by the constant-density acoustic equation);
 *   - the least-squares misfit J(v) with W_d = I (section 2) or the
 *     time-integral weighting of eq. (2);
 *   - the gradient dJ/dv by the adjoint-state method: zero-lag
 *     cross-correlation of the second time difference of the source wavefield
 *     with the back-propagated adjoint wavefield, times 2/v^3 (section 2; for
 *     eq. (2) the exact discrete counterpart of eq. (3));
 *   - the source-illumination pseudo-diagonal Hessian of eq. (1);
 *   - the diagonal part of the localized subsurface-offset Hessian of
 *     section 3, with the aperture factor of the Plessix-Mulder diagonal
 *     (section 1) standing in for the receiver-side Green's functions;
 *   - the gradient scaled by either diagonal (section 3.1, shot scaling and
 *     sub-offset Hessian scaling).
 *
 * Discretisation (the paper names only a time-domain finite-difference
 * engine): 8th-order 17-point Laplacian, leapfrog in time, an N-cell damping
 * sponge padded outside the model on all four sides (v edge-replicated),
 *   (1+g) u[n+1] = 2u[n] - (1-g) u[n-1] + dt^2 v^2 (L u[n] + f[n] e_src / h^2),
 * u[0] = u[-1] = 0, g = (dt/2) eta_max (d/N)^2, eta_max = 3 v_ref ln(1000)/(2 N h),
 * receivers record u[n] for n = 0 .. nt-1.  The gradient is taken with respect
 * to the model cells with the sponge padding held fixed.
 *
 * Conventions shared by every entry point
 *   - SI units; model grid [nz][nx], row-major, x contiguous, dz == dx.
 *   - Device pointers (v, wavelet, data, outputs, workspace) are caller-owned
 *     HIP device memory on the current device.  Geometry arrays inside
 *     fwi_geometry are HOST pointers; they are read during the call only.
 *   - The library never allocates device memory: all scratch lives in the
 *     caller's workspace, sized by fwi_workspace_bytes() (for
 *     fwi_offset_diag_exact by fwi_offset_diag_exact_workspace_bytes()).
 *   - Calls are asynchronous on `hip_stream` (a hipStream_t, NULL = default
 *     stream).  Do not run two calls concurrently on the same workspace.
 *   - Return 0 on success or a negative FWI_ERR_* code.  Every host-side check
 *     (arguments, geometry, CFL bound, workspace size) happens before anything
 *     is enqueued.  On error the outputs are unspecified; fwi_last_error()
 *     returns a thread-local message.  No C++ exception crosses the ABI.
 *   - Results are deterministic: repeated calls with the same inputs and
 *     execution settings are bitwise identical.
 */
#ifndef FWI_H
#define FWI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define FWI_OK              0
#define FWI_ERR_ARG        -1   /* null pointer, bad enum, non-positive size   */
#define FWI_ERR_GEOM       -2   /* source/receiver outside the model, bad CSR,
                                   nt[s] outside [2, nt_max], duplicate receiver
                                   cell within one shot                          */
#define FWI_ERR_CFL        -3   /* v_ref * dt / dx above the scheme's bound      */
#define FWI_ERR_WORKSPACE  -4   /* workspace smaller than fwi_workspace_bytes()  */
#define FWI_ERR_HIP        -5   /* a HIP runtime call failed                     */
#define FWI_ERR_NONFINITE  -6   /* (fwi_status) v non-finite, <= 0 or above the
                                   CFL bound on the device                       */
#define FWI_ERR_STATE      -7   /* fwi_misfit_backward without a matching
                                   fwi_misfit_forward in the same workspace      */

/* Stability bound of the scheme: v dt / h <= 2 / sqrt(2 * 6.50155). */
#define FWI_CFL_LIMIT 0.5546324796655889

/* ---------------------------------------------------------------- inputs */
/* dx, dt and v_ref are doubles: a time step such as 1 ms is not a float, and
 * a rounded dt enters every update through dt^2 v^2 / h^2 as a systematic
 * velocity bias (relative 1e-7) whose phase error grows with record length. */
typedef struct {
    int32_t nz, nx;     /* model cells (rows, columns)                         */
    double  dx;         /* grid spacing h in metres (dz == dx)                 */
    double  dt;         /* time step in seconds                                */
    int32_t nt_max;     /* trace length / stride of wavelet and data rows      */
    int32_t nsponge;    /* sponge width N in cells, >= 4                       */
    double  v_ref;      /* sponge reference velocity (m/s), also the declared
                           maximum velocity used for the CFL check             */
    int32_t free_surface; /* 0: sponge on all four sides.  1: pressure-free top
                           (the option of the scheme's reading with a free
                           surface): no sponge above the model, u = 0 on the
                           padded row just above model row 0 and the three
                           rows above it hold -u of the mirrored model rows
                           (antisymmetric image), for every wavefield        */
} fwi_grid;

typedef struct {
    int32_t nshot;              /* number of shots, >= 0                        */
    const int32_t *src_iz;      /* [nshot] source cell rows    (0 <= iz < nz)   */
    const int32_t *src_ix;      /* [nshot] source cell columns (0 <= ix < nx)   */
    const int32_t *rec_ptr;     /* [nshot+1] CSR: shot s owns receivers
                                   rec_ptr[s] .. rec_ptr[s+1]-1; rec_ptr[0] = 0 */
    const int32_t *rec_iz;      /* [rec_ptr[nshot]] receiver rows               */
    const int32_t *rec_ix;      /* [rec_ptr[nshot]] receiver columns            */
    const int32_t *nt;          /* [nshot] record length of each shot, 2..nt_max;
                                   NULL = nt_max for every shot                  */
} fwi_geometry;

/* Execution settings (all fields 0 = automatic). */
typedef struct {
    int32_t mode;             /* FWI_EXEC_BATCHED (default) or FWI_EXEC_PLAIN:
                                 plain = one shot at a time, one launch per
                                 time step, no graph, no autotuning            */
    int32_t shots_in_flight;  /* shots advanced together by one launch of the
                                 forward sweep                                 */
    int32_t tile_rows;        /* rows of one wavefront's tile (z sweep length)
                                 of the forward sweep                          */
    int32_t graph_steps;      /* time steps per captured hipGraph chunk;
                                 -1 = do not use graphs                        */
    int32_t autotune;         /* 1 = pick unset fields by timing a few steps
                                 of each candidate inside the call's workspace;
                                 the choice is cached per grid, geometry and
                                 GPU model in memory and, if the environment
                                 variable FWI_TUNE_CACHE names a file, in that
                                 file across processes; 0 = heuristic defaults */
    int32_t prefetch;         /* rows of loads a forward-sweep wavefront keeps
                                 in flight ahead of its z sweep: 1, 3 or 7     */
    int32_t prefetch_reverse; /* same for the fused reverse sweep: 1 or 3      */
    int32_t shots_in_flight_reverse; /* shots per launch of the reverse sweep;
                                 it takes each forward batch's shots this many
                                 at a time, so it must divide shots_in_flight
                                 (else the forward's value is used); for the
                                 autograd pair fwi_misfit_forward/backward,
                                 which keeps every shot's checkpoints, any
                                 value up to the number of shots (the shots,
                                 longest records first, this many at a time);
                                 0 = tuned, or the forward's                   */
    int32_t tile_rows_reverse; /* rows per tile of the reverse sweep; 0 =
                                 tuned, or tile_rows                           */
    int32_t reverse_steps;    /* time steps per launch of the adjoint sweep of
                                 fwi_gradient / fwi_misfit_backward /
                                 fwi_gn_hvp / fwi_extended_image: 1, or 2
                                 (temporal blocking: a workgroup computes the
                                 first step on 256 columns and the second on
                                 the 248 inside, one read and one write of
                                 every field for both); 0 = tuned, else 1.
                                 Two steps are not used with a free surface,
                                 in plain mode or for the eq. (3) variant      */
    int32_t forward_steps;    /* time steps per launch of the forward sweep
                                 of fwi_gradient / fwi_misfit_forward /
                                 fwi_extended_image: 1, or 2 (the same
                                 workgroup tiling; u[n+1], u[n+2], d[n+2]
                                 written once per two steps); 0 = tuned, else
                                 1.  Not used with a free surface, in plain
                                 mode, for Born modelling or the forward-only
                                 calls                                         */
    int32_t graph_branches;   /* independent launch chains that each captured
                                 chunk of the two-step sweeps is split into,
                                 each over a contiguous share of the launch's
                                 shots, so that one chain's launches run in
                                 the others' tails: 1 to 4 (at most the shots
                                 per launch); 0 = 2                            */
} fwi_exec;

enum { FWI_EXEC_BATCHED = 0, FWI_EXEC_PLAIN = 1 };
enum { FWI_MISFIT_L2 = 0,              /* section 2, W_d = I                   */
       FWI_MISFIT_TIME_INTEGRAL = 1,   /* eq. (2), W_d u = dt * running sum     */
       FWI_MISFIT_EQ3_LITERAL = 2 };   /* J of eq. (2), grad = eq. (3) taken
                                          literally (fwi_gradient only)         */
enum { FWI_HESS_EQ1 = 0,               /* eq. (1): H1 = sum_s E_s              */
       FWI_HESS_OFFSET = 1 };          /* offset diagonal D[2H+1][nz][nx]      */
enum { FWI_RCV_PM = 0,                 /* Plessix-Mulder aperture factor A_s   */
       FWI_RCV_NONE = 1 };             /* A_s = 1 (Shin form)                  */
enum { FWI_PRECOND_SHOT = 0,           /* P = (4/v^6) H1                       */
       FWI_PRECOND_OFFSET = 1 };       /* P = sum_h D(x, h)                    */
/* `what` argument of fwi_workspace_bytes */
enum { FWI_WS_FORWARD = 0, FWI_WS_GRADIENT = 1, FWI_WS_HESSIAN = 2,
       FWI_WS_AUTOGRAD = 3, FWI_WS_PRECOND = 4, FWI_WS_EXTIMAGE = 5,
       FWI_WS_BORN = 6, FWI_WS_GNHVP = 7 };

/* ---------------------------------------------------------------- sizing */
/* Bytes of device workspace needed by the matching entry point (hmax: offset
 * range of the offset diagonal, 0 if unused; for FWI_WS_EXTIMAGE the offset
 * range of the extended image, which sizes its buffers).  Returns 0 if the arguments fail
 * validation (see fwi_last_error).  FWI_WS_AUTOGRAD sizes the pair
 * fwi_misfit_forward / fwi_misfit_backward, which keeps the checkpoints of
 * every shot between the two calls. */
size_t fwi_workspace_bytes(const fwi_grid *grid, const fwi_geometry *geom,
                           const fwi_exec *exec, int what, int hmax);

/* The execution settings (shots_in_flight, tile_rows, graph_steps, prefetch,
 * prefetch_reverse, shots_in_flight_reverse, tile_rows_reverse,
 * reverse_steps, forward_steps, graph_branches) that a
 * call with these arguments uses: the autotuned choice once tuning has run on
 * the current device, else the heuristic defaults.  Fills *chosen (mode and
 * autotune copied from exec).  Returns 0 or FWI_ERR_*. */
int fwi_exec_query(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
                   int what, fwi_exec *chosen);

/* Host-side validation only (no HIP call).  Returns 0 or FWI_ERR_*. */
int fwi_validate(const fwi_grid *grid, const fwi_geometry *geom);

/* ---------------------------------------------------------------- compute */
/* Forward modelling (section 2, u synthesised by the acoustic equation).
 *   v        [nz][nx] float, m/s
 *   wavelet  [nshot][nt_max] float with row stride `wavelet_stride` floats;
 *            stride 0 = one wavelet shared by all shots
 *   data     [rec_ptr[nshot]][nt_max] float out: data[r][n] = u[n] at
 *            receiver r, zero for n >= nt[s]                                 */
int fwi_forward(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
                const float *v, const float *wavelet, int64_t wavelet_stride,
                float *data, void *workspace, size_t ws_bytes, void *hip_stream);

/* Misfit and gradient (section 2, eq. (2), eq. (3)).
 *   d_obs       [rec_ptr[nshot]][nt_max] recorded data (samples n >= nt[s]
 *               are ignored)
 *   misfit      FWI_MISFIT_L2 or FWI_MISFIT_TIME_INTEGRAL
 *   J           device double out: J = 1/2 sum (W_d r)^2 over shots,
 *               receivers and samples, r = synthetic - recorded
 *   grad        [nz][nx] float out: dJ/dv on model cells
 *   illum       [nz][nx] float out or NULL: H1 = sum_s sum_m (D_m/dt^2)^2 dt,
 *               D_m = u[m] - 2u[m-1] + u[m-2]   (eq. (1), time-domain form)
 *   offset_diag [2*hmax+1][nz][nx] float out or NULL: slice h + hmax holds
 *               D(x, h) = (4/v(x)^6) sum_s E_s(x + h) A_s(x - h), h in cells
 *               along x, terms leaving the model are 0 (section 3, diagonal
 *               part); rcv_model selects A_s                                  */
/* With misfit = FWI_MISFIT_EQ3_LITERAL, J is that of eq. (2) but grad is
 * eq. (3) taken literally -- u itself correlated with the adjoint of the
 * plain residual: grad = -(2/v^3) dt^2 sum_s sum_n u[n] lam_r[n+1].  It differs
 * from the exact eq. (2) gradient by an end-of-record term (the adjoint of
 * dt^2 sum_n r[n] injected at the last sample), which vanishes when every
 * residual trace integrates to zero. */
int fwi_gradient(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
                 const float *v, const float *wavelet, int64_t wavelet_stride,
                 const float *d_obs, int misfit,
                 double *J, float *grad, float *illum,
                 int hmax, int rcv_model, float *offset_diag,
                 void *workspace, size_t ws_bytes, void *hip_stream);

/* fwi_gradient without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same inputs, outputs and results as
 * fwi_gradient; the scratch lives in a static device array of
 * FWI_STATIC_SCRATCH_BYTES (64 MiB) per GPU, which the library holds until
 * the process ends.  The call allocates nothing: it runs direct launches
 * with the heuristic settings (exec's graph_steps and autotune are ignored,
 * its other fields apply) and returns FWI_ERR_WORKSPACE, before anything is
 * enqueued, when the call would need more scratch than the array holds (the
 * need is fwi_workspace_bytes(grid, geom, exec with graph_steps = -1 and
 * autotune = 0, FWI_WS_GRADIENT, hmax)).  Every call on one GPU uses that
 * GPU's one array and leaves its contents behind (each call sets up what it
 * reads): calls that overlap on one GPU -- on other streams or from other
 * threads -- race, and the caller must serialise them.  The device check of v
 * records its flag in that array, which fwi_status cannot read; a
 * non-finite or over-CFL v leaves the outputs unspecified. */
#define FWI_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int fwi_gradient_static(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
                        const float *v, const float *wavelet, int64_t wavelet_stride,
                        const float *d_obs, int misfit,
                        double *J, float *grad, float *illum,
                        int hmax, int rcv_model, float *offset_diag, void *hip_stream);

/* Offset-extended image: eq. (6) applied to the adjoint-state wavefields,
 * i.e. the gradient of J with respect to the extended model of eq. (5)
 * (section 3), for horizontal subsurface offsets h = -hmax .. hmax cells:
 *   image[h + hmax][z][x] = (2 / v(x)^3) sum_s sum_m lam_s[m](x - h) D_s[m](x + h)
 * with lam the adjoint wavefield of fwi_gradient and D_m = u[m] - 2u[m-1] +
 * u[m-2] of the source wavefield (receiver side at x - h, source side at
 * x + h); a term whose x - h or x + h leaves the model is 0.  The h = 0 slice
 * is dJ/dv.  Arguments as fwi_gradient; grad (NULL allowed) also receives
 * dJ/dv; image is [2*hmax+1][nz][nx] float, 0 <= hmax <= 32, hmax < nx.
 * Workspace: fwi_workspace_bytes(..., FWI_WS_EXTIMAGE, hmax); besides the
 * gradient's buffers it holds lam and D of the model cells for graph_steps
 * reverse steps per shot in flight (32 in plain mode). */
int fwi_extended_image(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
                       const float *v, const float *wavelet, int64_t wavelet_stride,
                       const float *d_obs, int misfit, double *J, float *grad,
                       int hmax, float *image,
                       void *workspace, size_t ws_bytes, void *hip_stream);

/* Born modelling (eq. (4)): the linearisation of fwi_forward in v along dv,
 * data = J dv.  The perturbation wavefield du obeys the scheme linearised at
 * the model cells (the sponge padding is frozen), starts from zero and in the
 * update that yields du[m] receives (2 dv / v) D[m], D[m] = u[m] - 2u[m-1] +
 * u[m-2]; data[r][n] = du[n] at receiver r.
 *   dv    [nz][nx] float, m/s
 *   data  [rec_ptr[nshot]][nt_max] float out, zero for n >= nt[s]
 * Workspace: fwi_workspace_bytes(..., FWI_WS_BORN, 0). */
int fwi_born(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
             const float *v, const float *wavelet, int64_t wavelet_stride,
             const float *dv, float *data,
             void *workspace, size_t ws_bytes, void *hip_stream);

/* Gauss-Newton Hessian-vector product (section 1, H = J^T J with the data
 * weighting W of the misfit): hv = J^T W^T W J dv on the model cells and
 * J = 1/2 |W J dv|^2 (device double), so that <dv, hv> = 2 J.  Runs Born
 * modelling (as fwi_born) with the source wavefield's checkpoints, takes the
 * Born data as the residual, and the adjoint sweep of fwi_gradient.
 *   misfit  FWI_MISFIT_L2 (W = I) or FWI_MISFIT_TIME_INTEGRAL (eq. (2))
 * Workspace: fwi_workspace_bytes(..., FWI_WS_GNHVP, 0). */
int fwi_gn_hvp(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
               const float *v, const float *wavelet, int64_t wavelet_stride,
               const float *dv, int misfit, double *J, float *hv,
               void *workspace, size_t ws_bytes, void *hip_stream);

/* The misfit J(v) alone (section 2 / eq. (2)), e.g. for line searches: the
 * forward sweep with recording and the misfit reduction, no checkpoints.
 * Arguments as fwi_gradient; J is a device double.
 * Workspace: fwi_workspace_bytes(..., FWI_WS_FORWARD, 0). */
int fwi_misfit_value(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
                     const float *v, const float *wavelet, int64_t wavelet_stride,
                     const float *d_obs, int misfit, double *J,
                     void *workspace, size_t ws_bytes, void *hip_stream);

/* Hessian diagonals from the forward wavefield alone (no adjoint pass).
 *   kind FWI_HESS_EQ1:    diag [nz][nx]            = H1            (eq. (1))
 *   kind FWI_HESS_OFFSET: diag [2*hmax+1][nz][nx]  = D(x, h)       (section 3) */
int fwi_hessian_diag(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
                     const float *v, const float *wavelet, int64_t wavelet_stride,
                     int kind, int hmax, int rcv_model, float *diag,
                     void *workspace, size_t ws_bytes, void *hip_stream);

/* The gradient split in two for reverse-mode differentiation of J(v).
 * fwi_misfit_forward runs the forward sweep of every shot, keeps each shot's
 * sqrt(nt) snapshots and per-step boundary strips in the workspace, and writes
 * J.  fwi_misfit_backward then runs the adjoint sweep from those checkpoints
 * and writes grad = (*grad_scale) dJ/dv (grad_scale: device double, NULL = 1)
 * plus the optional Hessian diagonals.  Both calls must receive the same
 * grid, geometry, exec, v, wavelet and workspace (FWI_WS_AUTOGRAD size);
 * otherwise fwi_misfit_backward returns FWI_ERR_STATE. */
int fwi_misfit_forward(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
                       const float *v, const float *wavelet, int64_t wavelet_stride,
                       const float *d_obs, int misfit, double *J,
                       void *workspace, size_t ws_bytes, void *hip_stream);
int fwi_misfit_backward(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
                        const float *v, const float *wavelet, int64_t wavelet_stride,
                        const double *grad_scale, float *grad, float *illum,
                        int hmax, int rcv_model, float *offset_diag,
                        void *workspace, size_t ws_bytes, void *hip_stream);

/* Diagonal of the subsurface-offset Hessian with the exact receiver term
 * (section 3: the diagonal part y = x, h_bar = h of the offset Hessian,
 * frequency by frequency, with the receiver Green's functions themselves in
 * place of the aperture factor that fwi_hessian_diag's FWI_HESS_OFFSET uses):
 *
 *   diag[h + hmax][z][x] = (4 / v^6) h_g^4 / (dt^4 L) sum_s sum_{r in R_s}
 *                          sum_k m_k |A_s(x + h, k)|^2 |B_r(x - h, k)|^2
 *
 * with L = 2 nt point DFTs (zero padded) of the discrete series
 *   A_s(y, j) = u[j+1] - 2 u[j] + u[j-1] at y (shot s, j = 0 .. nt-2),
 *   B_r(y, n) = u[n+1] at y of a run whose wavelet is [1, 0, 0, ...] with
 *               its source at receiver r (by reciprocity of the scheme, the
 *               response at r to a unit source term at y), n = 0 .. nt-2,
 * h_g the grid spacing, m_0 = 1, m_k = 2, and m = 1 for the Nyquist bin
 * k = nt.  fmax > 0 keeps the bins k <= fmax L dt (frequencies up to fmax
 * Hz); fmax = 0 keeps all nt + 1 of them (at most 65535 bins).  With every
 * bin this is the norm of the extended-Born column of (x, h) over the whole
 * response (conventional misfit).  Horizontal offsets |h| <= hmax <= 32;
 * terms with x+h or x-h outside the model are 0.
 *
 * Shots are grouped by (record length, receiver set); each group costs one
 * forward run per receiver and per shot, shots_in_flight runs at a time
 * (default 4 on grids of at least 1.5 M padded cells, else 8; of exec only
 * shots_in_flight, tile_rows and prefetch are used:
 * the sweeps are direct one-step launches, not graphs, and not autotuned).
 * A run's series are captured in FP32, 8192 / shots_in_flight updates at a
 * time (a multiple of 64, at least 64), and folded into its spectra by the
 * library's matrix-core kernel, the DFT matrix generated on chip from exact
 * phase tables: in FP32 (dft = FWI_DFT_FP32, v_mfma_f32_16x16x4_f32) or as
 * three bf16 products with FP32 accumulation of the series and the DFT
 * matrix split into bf16 pairs (FWI_DFT_BF16X3, v_mfma_f32_16x16x32_bf16:
 * about 16 significant bits per product, the lo*lo term dropped).  The
 * powers of a run's spectra are added to its side's sums by the kernel that
 * folds in its last chunk.  The workspace holds the chunks and spectra of
 * the runs in flight, the summed powers and the phase tables: see
 * fwi_offset_diag_exact_workspace_bytes (0 on bad arguments; the same for
 * both arithmetics).  Not with a free surface.  diag: device
 * [2 hmax + 1][nz][nx], overwritten. */
enum { FWI_DFT_FP32 = 0, FWI_DFT_BF16X3 = 1 };
size_t fwi_offset_diag_exact_workspace_bytes(const fwi_grid *grid, const fwi_geometry *geom,
                                             const fwi_exec *exec, int hmax, double fmax, int dft);
int fwi_offset_diag_exact(const fwi_grid *grid, const fwi_geometry *geom, const fwi_exec *exec,
                          const float *v, const float *wavelet, int64_t wavelet_stride,
                          int hmax, double fmax, int dft, float *diag,
                          void *workspace, size_t ws_bytes, void *hip_stream);

/* Preconditioned gradient (section 3.1): out = grad / (P + eps * max P) with
 * P = (4/v^6) * hdiag (kind SHOT, hdiag = H1 [nz][nx]) or
 * P = sum_h hdiag[h] (kind OFFSET, hdiag = D [2*hmax+1][nz][nx]).
 * workspace: at least fwi_workspace_bytes(..., FWI_WS_PRECOND, hmax) bytes. */
int fwi_precondition(const fwi_grid *grid, const float *v, const float *grad,
                     int kind, const float *hdiag, int hmax, float eps, float *out,
                     void *workspace, size_t ws_bytes, void *hip_stream);

/* Synchronises `hip_stream` and returns FWI_ERR_NONFINITE if the last call
 * that used this workspace found a non-finite, non-positive or over-CFL
 * velocity on the device (its outputs are then unspecified), else 0. */
int fwi_status(const void *workspace, void *hip_stream);

/* Forgets the autotuner's choices held in this process.  Later autotuned
 * calls read the FWI_TUNE_CACHE file again (if set) or tune again.  Must not
 * run concurrently with a call that is being autotuned. */
void fwi_tune_reset(void);

/* Thread-local description of the last error returned on this thread. */
const char *fwi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FWI_H */
