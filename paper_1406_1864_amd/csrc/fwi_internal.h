// Internal data layout shared by the host runtime and the gfx950 kernels of
// libfwi.  Nothing here is part of the public ABI.
//
// Storage of one padded field level (Z = nz + 2N rows, X = nx + 2N columns):
// row-major with pitch P floats; padded column x lives at storage column
// x + off, where `off` is chosen so that the model's first column (x = N)
// starts a 64-float (256-byte) line.  Storage columns outside [off, off + X)
// are held at zero and implement the zero boundary beyond the sponge; there
// are at least 4 of them on either side (off >= 4, P >= off + X + 4), and
// every wavefield level is followed by kGuardRows zero rows (the first level
// is also preceded by them).  A stencil load of a row or column just outside
// the grid therefore reads zeros from memory, without a test or a select.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace fwi {

constexpr int kWave = 64;         // CDNA wavefront width == tile width in x
constexpr int kWavesPerBlock = 4;  // independent wavefronts per workgroup
constexpr int kRadius = 4;         // stencil half-width (8th order)
// levels per checkpoint set of the source wavefield: u (two time levels) and
// the forward sweep's increment d[n] = u[n] - u[n-1]; the two-step reverse
// sweep adds a second pair of u levels (it reads one pair and writes the
// other), and likewise a second pair of adjoint levels
constexpr int kULevels = 3;
constexpr int kULevels2 = 5;
constexpr int kLamLevels = 2;
constexpr int kLamLevels2 = 4;
// two-step reverse sweep: a workgroup's 4 wavefronts compute the first step
// on 256 adjacent columns and the second on the 248 inside them; wave tile t
// starts at storage column off - 4 + kBlk2 (t / 4) + 64 (t % 4)
constexpr int kBlk2 = kWavesPerBlock * kWave - 2 * kRadius;
__host__ __device__ inline int tile2_x0(int off, int t) {
  return off - kRadius + kBlk2 * (t / kWavesPerBlock) + kWave * (t % kWavesPerBlock);
}
// zero rows after each wavefield level (and before the first one): covers the
// sweep's loads of rows -4 - 1 .. Z - 1 + 4 + 7 + 1 (stencil reach, the
// longest prefetch and a halo column wrapping into the next row)
constexpr int kGuardRows = 16;

struct Dims {
  int32_t nz, nx, N;     // model rows / columns, sponge width
  int32_t Z, X;          // padded rows / columns
  int32_t P, off;        // storage pitch (floats) and column offset
  int32_t mx0;           // storage column of model column 0 (multiple of 64)
  int32_t XT, ZT, TZ;    // wave tiles along x and z, rows per tile
  int32_t ring;          // floats of one boundary-strip ring: 8 (nx + nz)
  int32_t fs;            // free surface: rows above the model mirror it (odd image)
  int32_t ztop;          // first computed padded row: N with a free surface, else 0
  int64_t field;         // floats per field level: (Z + kGuardRows) * P
  int64_t guard;         // floats of the guard rows: kGuardRows * P
  int64_t model;         // floats per model-grid array: nz * nx
};

struct ShotDesc {
  int32_t nt;          // record length
  int32_t K;           // snapshot spacing
  int32_t nsnap;       // snapshot pairs kept
  int32_t src_z;       // padded row of the source cell
  int32_t src_xs;      // storage column of the source cell
  int32_t rec_begin;   // first global trace index of the shot
  int32_t nrec;        // receivers of the shot
  int32_t rdir;        // first receiver-map directory entry (one per x tile)
  int32_t rec_z0;      // shallowest receiver row (model rows)
  float xmin_m, xmax_m;  // receiver aperture in metres
  int32_t rdir2;       // first directory entry of the two-step reverse tiling
};

struct SlotInfo {
  int32_t shot;  // shot index or -1 (idle slot)
  int32_t cs;    // checkpoint set: index of the u fields / snapshots / strips
};

struct RmapDir { int32_t begin, count; };  // per (shot, x tile): rows in RmapRow
struct RmapRow { int32_t z, map; };         // padded row; offset of a 64-entry map

// Kernel arguments of one time step over a batch of shots.
struct StepArgs {
  Dims d;
  int32_t S;            // slots in the launch
  int32_t xcd_map;      // 1: keep each slot's tiles on one XCD
  const SlotInfo* slots;
  const ShotDesc* shots;
  const RmapDir* rdir;   // receiver maps of the launch's tiling (the two-step
  const RmapRow* rrows;  // reverse sweep has tiles of its own)
  const int32_t* rmaps;
  const float* w;       // dt^2 v^2 / h^2 on the padded grid (storage layout)
  float* u;             // [cs][ulevels][field]: u[n] at level n & 1, increment at 2
  float* lam;           // [slot][lamlevels][field] adjoint wavefield
  int64_t ustride;      // floats per checkpoint set of u (ulevels * field)
  int64_t lstride;      // floats per slot of lam (lamlevels * field)
  float* g;             // [slot][model]    sum_m lam[m] D[m]
  float* E;             // [slot][model]    sum_m D[m]^2
  float* traces;        // [nt_max][ntrace] recorded u (forward) / psi' (adjoint)
  int32_t ntrace;
  const float* wavelet;
  int64_t wstride;
  float* snap;          // [cs] blocks of snap_stride floats: [nsnap][2][model]
  float* strip;         // [cs] blocks of strip_stride floats: [nt][ring]
  int64_t snap_stride, strip_stride;
  double sp_a;          // sponge damping g = sp_a * d^2 (d: cells into sponge)
  const int32_t* step_ctr;  // device step base (graph replay) or null
  int32_t step;             // step offset, or absolute step if step_ctr is null
  const int32_t* err;       // device error flag: nonzero = skip all work
  // extended imaging (reverse sweep only): lam[m] and D[m] of the model cells
  // are kept for the last ext_T launch steps, ring slot = step % ext_T
  float* ext_lam;       // [slot][ext_T][model]
  float* ext_D;         // [slot][ext_T][model]
  int32_t ext_T;
  // Born modelling (forward sweep only): the perturbation wavefield
  float* bu;            // [cs][3][field]  du[n] at level n & 1, its increment at level 2
  const float* bw;      // 2 dv / v on the padded grid (zero outside the model)
  // series capture (forward sweep, kFwdCapD / kFwdCapU): the value of
  // update n of model cell `cell` (row-major model index) goes, as FP32, to
  // element (slot * cap_T + n - cap_n0) * cap_R + cell of cap: per slot a
  // chunk of cap_T updates, time-major, cap_R >= nz nx cells per row
  float* cap;
  int64_t cap_R;
  int32_t cap_n0, cap_T;
};

// Extended imaging over one window of reverse launch steps
// [base + step0, base + step0 + count), base = *step_ctr (or 0):
//   I(x, h) += sum_slots sum_steps lam[m](x - h) D[m](x + h)
struct ExtArgs {
  Dims d;
  int32_t S;
  const SlotInfo* slots;
  const ShotDesc* shots;
  const float* lam;     // [slot][T][model]
  const float* D;       // [slot][T][model]
  int32_t T;
  float* I;             // [groups][2 hmax + 1][model]: one partial sum per slot group
  int32_t hmax;
  int32_t groups;       // slots are split into this many groups (parallelism)
  const int32_t* step_ctr;  // launches done (graph replays), or null
  int32_t step_mul;         // reverse steps per launch: the window starts at step_mul * *step_ctr + step0
  int32_t step0, count;     // in reverse steps
  const int32_t* err;
};

// reverse-kernel variants: kRevExt keeps lam and D for extended imaging;
// kRevImgU correlates lam[m] with u[m-1] instead of D[m] (eq. (3) taken literally)
enum : int { kRevExt = 1, kRevImgU = 2 };

// forward-kernel feature flags
// kFwdBorn: also step the Born perturbation wavefield and record it instead of u
// (kFwdFS, the free-surface variant, is chosen by the launcher from Dims::fs)
// kFwdCapD / kFwdCapU: capture D[n+1] = u[n+1] - 2u[n] + u[n-1] (resp. u[n+1])
// of the model cells at every update (StepArgs::cap)
enum : int { kFwdRecord = 1, kFwdCkpt = 2, kFwdIllum = 4, kFwdBorn = 8, kFwdFS = 16, kFwdCapD = 32, kFwdCapU = 64 };

struct MisfitArgs {
  const SlotInfo* slots;
  const ShotDesc* shots;
  float* traces;        // in: recorded synthetic u (time-major); out: psi'
  const float* dobs;    // [ntrace][nt_max]
  int32_t ntrace, nt_max, kind;
  double dt, psi_scale;
  double* Jpart;        // [ntrace]
  const int32_t* err;
};

struct EpiArgs {
  Dims d;
  int32_t S;
  const SlotInfo* slots;
  const ShotDesc* shots;
  const float* E;       // [slot][model]
  const float* v;       // [nz][nx]
  float* H1;            // [nz][nx] or null
  float* D;             // [2H+1][nz][nx] or null
  int32_t hmax, rcv_none;
  float h, inv_dt3;
  const int32_t* err;
};

// host-side launchers (fwi_kernels.hip)
hipError_t launch_prep(const Dims& d, const float* v, float* w, double dt, double h, float vmax,
                       int32_t* err, hipStream_t s);
hipError_t launch_fill(void* p, size_t nbytes, hipStream_t s);
// bw = 2 dv / v on the model cells of the padded grid (storage layout), 0 elsewhere
hipError_t launch_prep_born(const Dims& d, const float* v, const float* dv, float* bw, hipStream_t s);
hipError_t launch_fill_slots(float* base, int64_t stride, int64_t count, const SlotInfo* slots,
                             int S, int use_cs, hipStream_t s);
// prefetch: rows of loads in flight ahead of the sweep (forward 1, 3, 7; reverse 1, 3)
hipError_t launch_forward(const StepArgs& a, int flags, int prefetch, hipStream_t s);
// flags: 0, kRevExt (StepArgs::ext_* set) or kRevImgU
hipError_t launch_reverse(const StepArgs& a, int prefetch, int flags, hipStream_t s);
hipError_t launch_ext_image(const ExtArgs& a, hipStream_t s);
// two reverse steps per launch (StepArgs::d.XT = two-step tiles, receiver
// maps of that tiling, step = launch index); no extended image, eq. (3) or
// free surface
hipError_t launch_reverse2(const StepArgs& a, int prefetch, int flags, hipStream_t s);
hipError_t launch_forward2(const StepArgs& a, int prefetch, hipStream_t s);
// after a two-step forward sweep: shots whose final state sits in the second
// set of u levels (an odd number of launches) get it copied to the first
hipError_t launch_forward2_finish(float* u, int64_t ustride, int64_t set_floats, const SlotInfo* slots,
                                  const ShotDesc* shots, int S, hipStream_t s);
hipError_t launch_ext_out(const Dims& d, const float* Iacc, int groups, int hmax, const float* v, float* image,
                          const int32_t* err, hipStream_t s);
hipError_t launch_advance(int32_t* ctr, int32_t by, hipStream_t s);
hipError_t launch_set(int32_t* ctr, int32_t value, hipStream_t s);
hipError_t launch_misfit(const MisfitArgs& a, int S, int max_nrec, hipStream_t s);
hipError_t launch_reduce_J(const double* part, int n, double* J, const int32_t* err, hipStream_t s);
hipError_t launch_epilogue(const EpiArgs& a, hipStream_t s);
// grad = fac * scale * (2/v^3) * sum over slots
hipError_t launch_gradient_out(const Dims& d, const float* gacc, int S, const float* v,
                               const double* scale, double fac, float* grad, const int32_t* err, hipStream_t s);
hipError_t launch_traces_out(const float* traces, int ntrace, int nt_max, const ShotDesc* shots,
                             const int32_t* trace_shot, float* data, hipStream_t s);
// exact offset diagonal: spectra of the captured series on the matrix cores
// (fwi_dft.hip).  A workgroup owns kDftCols columns of the DFT matrix (the
// cosine and sine rows of kDftCols / 2 bins) by kDftCells model cells and
// walks the time steps kDftKT at a time.
constexpr int kDftCols = 256;
constexpr int kDftCells = 256;
constexpr int kDftKT = 32;

struct DftArgs {
  const float* X;       // captured series [slot][Tc][R], FP32, time-major
  int64_t R;            // cells per series row: ntile * kDftCells >= model
  int64_t xslot;        // floats per slot of X (Tc * R)
  int32_t tc;           // valid steps of this chunk: rows t >= tc count as 0
  int32_t nslab;        // slabs of kDftKT steps in the chunk: ceil(tc / kDftKT)
  const float2* Tb;     // [Kp][kDftKT] (cos, sin)(2 pi k tau / L)       (launch_dft_tables)
  const float2* Ph;     // [slab][Kp]   (cos, sin)(2 pi k 32 slab / L)
  int32_t Kp;           // bins of the tables: Cp / 2
  int32_t j0;           // the chunk's first slab (absolute)
  int32_t Cp;           // columns of the DFT matrix and of C: 2K rounded up to kDftCols
  float* C;             // running spectra [slot][Cp][R] (not read when first,
                        // not written when last)
  int32_t first, last;  // the run's first / last chunk
  float* P;             // [Kp][R]: last chunk adds C[2k]^2 + C[2k+1]^2 of every slot
  int32_t K;
  int64_t model;
  int32_t nslots;       // runs of the launch (slots 0 .. nslots-1)
  int32_t ntile;        // cell tiles
};
// split: bf16 hi/lo operands (three products, FP32 accumulation); else FP32
hipError_t launch_dft(const DftArgs& a, int split, hipStream_t s);
// the phase tables of the DFT matrix w(t, c) = cos / sin (2 pi k t / L),
// c = 2k / 2k + 1: Tb[k][tau] for tau < kDftKT and Ph[J][k] for the slabs'
// first steps t = kDftKT J, J < nslab; (cos, sin) with the phase k t mod L
// reduced exactly in integers, zero for k >= K
hipError_t launch_dft_tables(float2* Tb, float2* Ph, int nslab, int Kp, int K, int L, hipStream_t s);
// D[h][z][x] += scale / v^6 sum_k m_k PA[k][z][x+h] PB[k][z][x-h] for |h| <= hmax
// (both columns in the model), m_0 = 1, m_{K-1} = 1 if nyq, else 2; bin k
// of PA / PB starts at element k * ldp
hipError_t launch_diag_products(const float* PA, const float* PB, int64_t ldp, int K, int nyq, int nz, int nx,
                                int hmax, const float* v, float scale, float* D, const int32_t* err,
                                hipStream_t s);
hipError_t launch_precond(int nz, int nx, const float* v, const float* grad, int kind,
                          const float* hdiag, int hmax, float eps, float* out, uint32_t* maxbits,
                          hipStream_t s);

}  // namespace fwi
