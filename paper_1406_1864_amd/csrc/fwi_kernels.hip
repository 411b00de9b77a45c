// gfx950 kernels of libfwi: 2D acoustic 8th-order/leapfrog time stepping
// with the fused adjoint-state gradient and Hessian-diagonal accumulations.
//
// Method: Huang, Wang & Ren, "Two new gradient precondition schemes for full
// waveform inversion" -- section 2 (least-squares misfit, zero-lag
// cross-correlation gradient scaled by 2/v^3), eq. (2) and eq. (3) (the
// time-integral misfit and its adjoint-state gradient), eq. (1) (source
// illumination pseudo-diagonal Hessian) and section 3 (diagonal part of the
// subsurface-offset Hessian).  The discrete scheme is stated in include/fwi.h.
//
// Execution model (memory-bound stencil, no MFMA):
//   * one wavefront owns a 64-column tile of one shot and sweeps it along z,
//     keeping the 9 rows of the vertical stencil in registers (register
//     sliding); the +-4 horizontal neighbours come from a per-wavefront LDS
//     row with a 4-column halo on each side;
//   * a launch advances every shot of a batch by one time step; a block holds
//     4 independent wavefronts (no block barrier), and with 8k shots in the
//     batch all tiles of a shot stay on one XCD, so stencil halos are re-read
//     from that XCD's L2;
//   * interior cells use an FP32 difference-form Laplacian
//     sum_k c_k ((neighbours at distance k) - 4u) and one FMA update; sponge
//     cells are updated in FP64 (the damping coefficients are the error
//     source of an all-FP32 scheme).  Fields stay FP32 in HBM.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>

#include <algorithm>
#include <utility>

#include "fwi_internal.h"

namespace fwi {

// 8th-order second-derivative weights c1..c4 (c0 = -4 * (c1+..+c4)/2 folded
// into the difference form)
constexpr float kC1 = 8.0f / 5.0f;
constexpr float kC2 = -1.0f / 5.0f;
constexpr float kC3 = 8.0f / 315.0f;
constexpr float kC4 = -1.0f / 560.0f;

__device__ __forceinline__ float ck(int k) {
  return k == 1 ? kC1 : (k == 2 ? kC2 : (k == 3 ? kC3 : kC4));
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// f(integral_constant<int, 0>) ... f(integral_constant<int, N-1>): a loop
// unrolled by construction, whatever the size of its body (register rings
// indexed by the loop counter need every index to be a constant)
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Wavefront-local LDS exchange: LDS operations of one wavefront complete in
// program order, so only compiler reordering has to be prevented.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// blockIdx/wave -> (slot, tile).  Tiles of one slot are numbered x-fastest.
__device__ __forceinline__ bool map_tile(const Dims& d, int S, int xcd_map, int wave,
                                         int& slot, int& tile) {
  const int T = d.XT * d.ZT;
  const int bps = (T + kWavesPerBlock - 1) / kWavesPerBlock;
  const int b = blockIdx.x;
  int tb;
  if (xcd_map) {
    // consecutive block ids go to consecutive XCDs: give XCD c the slots
    // c, c+8, c+16, ... so that neighbouring tiles share one L2
    const int xcd = b & 7, r = b >> 3;
    slot = (r / bps) * 8 + xcd;
    tb = r % bps;
  } else {
    slot = b / bps;
    tb = b % bps;
  }
  tile = tb * kWavesPerBlock + wave;
  return slot < S && tile < T;
}

__device__ __forceinline__ int step_of(const StepArgs& a) {
  return a.step_ctr ? (*a.step_ctr + a.step) : a.step;
}

// Per-lane column classification of a wavefront tile (computed once).
struct Col {
  int xs;      // storage column
  int x;       // padded column
  bool xin;    // inside the padded grid
  int dxs;     // cells into the sponge along x (0 inside the model columns)
  int mx;      // model column (valid if mcol)
  bool mcol;   // model column
  int side;    // strip index base of a left/right ring column, -1 otherwise
  int hcol;    // halo column held by lanes 0..7
  bool hok;    // this lane loads a halo value
  int hsafe;   // column a lane's halo load reads: hcol (lanes 0..7), else its own column
  int mxc;     // model column clamped into [0, nx): in-bounds model-grid loads
};

__device__ __forceinline__ Col make_col(const Dims& d, int xs0, int lane) {
  Col c;
  c.xs = xs0 + lane;
  c.x = c.xs - d.off;
  c.xin = c.x >= 0 && c.x < d.X;
  c.dxs = max(max(d.N - c.x, c.x - (d.N + d.nx - 1)), 0);
  c.mx = c.xs - d.mx0;
  c.mcol = c.mx >= 0 && c.mx < d.nx;
  c.side = (c.mx >= -kRadius && c.mx < 0) ? 8 * d.nx + (c.mx + kRadius)
           : (c.mx >= d.nx && c.mx < d.nx + kRadius) ? 8 * d.nx + 4 * d.nz + (c.mx - d.nx) : -1;
  c.hcol = lane < 4 ? xs0 - 4 + lane : xs0 + 60 + lane;
  c.hok = lane < 8 && c.hcol >= 0 && c.hcol < d.P;
  c.hsafe = lane < 8 ? c.hcol : c.xs;
  c.mxc = min(max(c.mx, 0), d.nx - 1);
  return c;
}

// Free surface: a row above the model reads the odd image of the model rows
// about padded row N-1 (itself never written, so it stays 0).  Returns the
// row to load and its sign.
__device__ __forceinline__ int image_row(const Dims& d, int r, float& sg) {
  sg = 1.0f;
  if (d.fs && r < d.N - 1) {
    sg = -1.0f;
    return 2 * (d.N - 1) - r;
  }
  return r;
}

// row index clamped into the padded grid, for loads issued whatever the row
__device__ __forceinline__ int clamp_row(const Dims& d, int r) { return min(max(r, 0), d.Z - 1); }

// Uniform classification of one padded row.
struct Row {
  int mz;      // model row
  bool model;  // model row
  int dz;      // cells into the sponge along z
  int tb;      // strip index base of a top/bottom ring row, -1 otherwise
};

__device__ __forceinline__ Row make_row(const Dims& d, int z) {
  Row r;
  r.mz = z - d.N;
  r.model = r.mz >= 0 && r.mz < d.nz;
  r.dz = max(max(-r.mz, r.mz - (d.nz - 1)), 0);
  r.tb = (r.mz >= -kRadius && r.mz < 0) ? (r.mz + kRadius) * d.nx
         : (r.mz >= d.nz && r.mz < d.nz + kRadius) ? 4 * d.nx + (r.mz - d.nz) * d.nx : -1;
  return r;
}

// strip index of cell (row, col) of the 4-cell ring around the model, or -1
__device__ __forceinline__ int strip_index(const Row& r, const Col& c) {
  if (r.model) return c.side >= 0 ? c.side + 4 * r.mz : -1;
  return (r.tb >= 0 && c.mcol) ? r.tb + c.mx : -1;
}

// 8th-order Laplacian (times h^2) in difference form from the register
// window (z neighbours) and the wavefront's LDS row (x neighbours).
template <int W>
__device__ __forceinline__ float laplace(const float (&win)[W], int ctr, const float* lds, int lane) {
  const float c = win[ctr % W];
  float lap = 0.0f;
#pragma unroll
  for (int k = 4; k >= 1; --k) {
    const float sz = win[(ctr - k + W) % W] + win[(ctr + k) % W];
    const float sx = lds[kRadius + lane - k] + lds[kRadius + lane + k];
    lap = fmaf(ck(k), fmaf(-4.0f, c, sz + sx), lap);
  }
  return lap;
}

__device__ __forceinline__ void lds_put(float* lds, int lane, float c, float h) {
  lds[kRadius + lane] = c;
  if (lane < 4) lds[lane] = h;
  else if (lane < 8) lds[kWave + lane] = h;
}

// FP64 damped update of a sponge cell: ((2c - (1-g) p + w lap) / (1+g))
__device__ __forceinline__ float sponge_update(double sp_a, int dd, float c, float p, float w, float lap) {
  const double gm = sp_a * (double)(dd * dd);
  return (float)((2.0 * (double)c - (1.0 - gm) * (double)p + (double)w * (double)lap) / (1.0 + gm));
}

// -------------------------------------------------------------------------
// forward step n -> n+1 for every shot of the batch, in increment form:
//   d[n+1] = ((1-g) d[n] + w (L u[n] + f[n] e_src)) / (1+g),  u[n+1] = u[n] + d[n+1]
// with d[n] = u[n] - u[n-1] kept as its own FP32 state (in place).  This is
// the leapfrog update rearranged; rounding u[n+1] no longer perturbs the
// velocity d, which makes the recorded traces ~3x more accurate than the
// two-level form at 4 more bytes per update.  u[n+1] overwrites u[n-1], so the
// two u levels hold exactly what the reverse sweep expects.
// The z sweep keeps W = 9 + PF rows of u[n] in registers and issues the loads
// of row z+4+PF (and the point-wise operands of row z+PF) PF rows ahead, so
// several rows of loads are in flight per wavefront.
// -------------------------------------------------------------------------
template <int FLAGS, int PF>
__global__ __launch_bounds__(256) void k_forward(StepArgs a) {
  constexpr int W = 9 + PF;  // stencil-row ring
  constexpr int R = PF + 1;  // point-wise ring; W % R == 0 keeps slots static
  static_assert(W % R == 0, "prefetch distance must make the rings commensurate");
  constexpr bool BORN = (FLAGS & kFwdBorn) != 0;
  constexpr bool FS = (FLAGS & kFwdFS) != 0;
  __shared__ float lds_all[kWavesPerBlock][kWave + 2 * kRadius];
  __shared__ float ldsB_all[kWavesPerBlock][BORN ? kWave + 2 * kRadius : 1];
  const int lane = threadIdx.x & 63;
  const int wv = uniform(threadIdx.x >> 6);
  int slot, tile;
  if (!map_tile(a.d, a.S, a.xcd_map, wv, slot, tile)) return;
  if (*a.err) return;
  const SlotInfo si = a.slots[slot];
  if (si.shot < 0) return;
  const ShotDesc sd = a.shots[si.shot];
  const int n = step_of(a);
  if (n >= sd.nt - 1) return;

  const Dims& d = a.d;
  float* lds = lds_all[wv];
  const int xt = tile % d.XT, zt = tile / d.XT;
  const int xs0 = xt * kWave;
  const Col col = make_col(d, xs0, lane);
  const int z0 = (FS ? d.ztop : 0) + zt * d.TZ, z1 = min(z0 + d.TZ, d.Z);
  float* ubase = a.u + (int64_t)si.cs * a.ustride;
  const float* ucur = ubase + (int64_t)(n & 1) * d.field;
  float* unxt = ubase + (int64_t)((n + 1) & 1) * d.field;
  float* dinc = ubase + (int64_t)2 * d.field;
  // Born: du with the same level layout as u
  float* bbase = BORN ? a.bu + (int64_t)si.cs * kULevels * d.field : nullptr;
  const float* bcur = BORN ? bbase + (int64_t)(n & 1) * d.field : nullptr;
  float* bnxt = BORN ? bbase + (int64_t)((n + 1) & 1) * d.field : nullptr;
  float* binc = BORN ? bbase + (int64_t)2 * d.field : nullptr;
  float* ldsB = ldsB_all[wv];

  const bool src_tile = sd.src_z >= z0 && sd.src_z < z1 && sd.src_xs >= xs0 && sd.src_xs < xs0 + kWave;
  const float fsrc = src_tile ? a.wavelet[(int64_t)si.shot * a.wstride + n] : 0.0f;

  // tiles of even zt sweep down (increasing z), odd ones up: two vertically
  // neighbouring tiles then read the rows they share at about the same time
  // (the second read comes from L2); the top tile of a free-surface grid
  // (zt = 0) always sweeps down
  const int dz = (zt & 1) ? -1 : 1;
  const int zS = dz > 0 ? z0 : z1 - 1, nT = z1 - z0;
  int rp = 0, rbeg = 0, rend = 0, rz = INT_MAX;
  if (FLAGS & kFwdRecord) {
    const RmapDir dir = a.rdir[sd.rdir + xt];
    rbeg = dir.begin;
    rend = dir.begin + dir.count;
    if (dz > 0) {
      rp = rbeg;
      while (rp < rend && a.rrows[rp].z < z0) ++rp;
    } else {
      rp = rend - 1;
      while (rp >= rbeg && a.rrows[rp].z >= z1) --rp;
    }
    rz = (rp >= rbeg && rp < rend) ? a.rrows[rp].z : INT_MAX;
  }
  // snapshot pair k holds (u[a_k], u[a_k - 1]) with a_k = nt-1-kK, k >= 1
  bool save = false;
  float *snap0 = nullptr, *snap1 = nullptr, *strip = nullptr;
  if (FLAGS & kFwdCkpt) {
    const int rem = sd.nt - 2 - n;  // nt-1 - (n+1)
    save = rem > 0 && (rem % sd.K) == 0;
    if (save) {
      snap0 = a.snap + (int64_t)si.cs * a.snap_stride + (int64_t)(rem / sd.K - 1) * 2 * d.model;
      snap1 = snap0 + d.model;
    }
    strip = a.strip + (int64_t)si.cs * a.strip_stride + (int64_t)(n + 1) * d.ring;
  }
  float* E = (FLAGS & kFwdIllum) ? a.E + (int64_t)slot * d.model : nullptr;

  float wc[W], wh[W], pd[R], pw[R];
  float bc[BORN ? W : 1], bh[BORN ? W : 1], pbd[BORN ? R : 1], pbw[BORN ? R : 1];
  // rows and halo columns just outside the grid read the zero guard rows and
  // columns of the layout; the point-wise operands of rows past the grid are
  // loaded from its last row and never used
  auto load_row = [&](int r, float& c, float& h) {
    const float* row = ucur + (int64_t)r * d.P;
    c = row[col.xs];
    h = row[col.hsafe];
  };
  auto load_brow = [&](int r, float& c, float& h) {
    const float* row = bcur + (int64_t)r * d.P;
    c = row[col.xs];
    h = row[col.hsafe];
  };
  auto load_pt = [&](int r, float& p, float& w) {
    const int64_t idx = (int64_t)clamp_row(d, r) * d.P + col.xs;
    p = dinc[idx];
    w = a.w[idx];
  };
  auto load_bpt = [&](int r, float& p, float& f) {
    const int64_t idx = (int64_t)clamp_row(d, r) * d.P + col.xs;
    p = binc[idx];
    f = a.bw[idx];
  };
  // Only the first window of the top tile reaches above the model; with a
  // free surface it reads the odd image there.  Elsewhere the loads are issued
  // back to back and consumed later in the sweep.
  if (FS && z0 == d.ztop) {
#pragma unroll
    for (int j = 0; j < 8 + PF; ++j) {
      float sg;
      const int r = image_row(d, z0 - 4 + j, sg);
      load_row(r, wc[j], wh[j]);
      wc[j] *= sg;
      wh[j] *= sg;
      if (BORN) {
        load_brow(r, bc[j % (BORN ? W : 1)], bh[j % (BORN ? W : 1)]);
        bc[j % (BORN ? W : 1)] *= sg;
        bh[j % (BORN ? W : 1)] *= sg;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8 + PF; ++j) {
      load_row(zS + dz * (j - 4), wc[j], wh[j]);
      if (BORN) load_brow(zS + dz * (j - 4), bc[j % (BORN ? W : 1)], bh[j % (BORN ? W : 1)]);
    }
  }
#pragma unroll
  for (int j = 0; j < PF; ++j) {
    load_pt(zS + dz * j, pd[j], pw[j]);
    if (BORN) load_bpt(zS + dz * j, pbd[j % (BORN ? R : 1)], pbw[j % (BORN ? R : 1)]);
  }

  // sweep position j is row zS + dz j; the rings hold positions, and the
  // stencil is symmetric in z
  for (int jb = 0; jb < nT; jb += W) {
#pragma unroll
    for (int r = 0; r < W; ++r) {
      const int j = jb + r;
      if (j >= nT) break;
      const int z = zS + dz * j;
      // the next rows' loads are issued on every row, also past the tile
      // (clamped into the grid): with the same loads on every path the
      // compiler waits only for the rows consumed now
      load_row(z + dz * (4 + PF), wc[(r + 8 + PF) % W], wh[(r + 8 + PF) % W]);
      load_pt(z + dz * PF, pd[(r + PF) % R], pw[(r + PF) % R]);
      if (BORN) {
        load_brow(z + dz * (4 + PF), bc[(r + 8 + PF) % (BORN ? W : 1)], bh[(r + 8 + PF) % (BORN ? W : 1)]);
        load_bpt(z + dz * PF, pbd[(r + PF) % (BORN ? R : 1)], pbw[(r + PF) % (BORN ? R : 1)]);
      }
      const float c = wc[(r + 4) % W];
      lds_put(lds, lane, c, wh[(r + 4) % W]);
      float bcv = 0.0f;
      if (BORN) {
        bcv = bc[(r + 4) % (BORN ? W : 1)];
        lds_put(ldsB, lane, bcv, bh[(r + 4) % (BORN ? W : 1)]);
      }
      wave_lds_fence();
      float lap = laplace<W>(wc, r + 4, lds, lane);
      float blap = 0.0f;
      if (BORN) blap = laplace<BORN ? W : 1>(bc, r + 4, ldsB, lane);
      wave_lds_fence();
      if (src_tile && z == sd.src_z && col.xs == sd.src_xs) lap += fsrc;

      const Row row = make_row(d, z);
      const float dn = pd[r % R], wv_ = pw[r % R];
      float out = 0.0f, bout = 0.0f;
      if (col.xin) {
        const int dd = max(row.dz, col.dxs);
        float dnew, bdnew = 0.0f;
        if (dd == 0) {
          dnew = fmaf(wv_, lap, dn);
          // Born: d(du) = w (L du + (2 dv / v)(L u + s)), the linearised update
          if (BORN) bdnew = fmaf(wv_, fmaf(pbw[r % (BORN ? R : 1)], lap, blap), pbd[r % (BORN ? R : 1)]);
        } else {
          const double gm = a.sp_a * (double)(dd * dd);
          dnew = (float)(((1.0 - gm) * (double)dn + (double)wv_ * (double)lap) / (1.0 + gm));
          if (BORN)
            bdnew = (float)(((1.0 - gm) * (double)pbd[r % (BORN ? R : 1)] + (double)wv_ * (double)blap) /
                            (1.0 + gm));
        }
        out = c + dnew;
        const int64_t idx = (int64_t)z * d.P + col.xs;
        unxt[idx] = out;
        dinc[idx] = dnew;
        if (BORN) {
          bout = bcv + bdnew;
          bnxt[idx] = bout;
          binc[idx] = bdnew;
        }
        const bool mcell = row.model && col.mcol;
        const int64_t mi = (int64_t)row.mz * d.nx + col.mx;
        if ((FLAGS & kFwdIllum) && mcell) {
          const float D = wv_ * lap;
          E[mi] = (n == 0) ? D * D : fmaf(D, D, E[mi]);
        }
        if ((FLAGS & (kFwdCapD | kFwdCapU)) && mcell)
          a.cap[((int64_t)slot * a.cap_T + (n - a.cap_n0)) * a.cap_R + mi] = (FLAGS & kFwdCapD) ? wv_ * lap : out;
        if (FLAGS & kFwdCkpt) {
          const int ri = strip_index(row, col);
          if (ri >= 0) strip[ri] = out;
          if (save && mcell) {
            snap0[mi] = out;
            snap1[mi] = c;
          }
        }
      }
      if (FLAGS & kFwdRecord) {
        if (z == rz) {
          const int tr = a.rmaps[a.rrows[rp].map + lane];
          if (tr >= 0) a.traces[(int64_t)(n + 1) * a.ntrace + tr] = BORN ? bout : out;
          rp += dz;
          rz = (rp >= rbeg && rp < rend) ? a.rrows[rp].z : INT_MAX;
        }
      }
    }
  }
}

// -------------------------------------------------------------------------
// reverse step m (= nt-1-j for global reverse step j), fused:
//   u[m-2] = 2u[m-1] - u[m] + w (L u[m-1] + f[m-1] e_src)   (model cells)
//   strip ring of u[m-2] restored from the forward's boundary strips
//   lam[m] = damped leapfrog of lam[m+1], lam[m+2] + w psi'[m] at receivers
//   g += lam[m] D[m],  E += D[m]^2,  D[m] = w (L u[m-1] + f[m-1] e_src)
// Same register sweep and prefetch as the forward, for two fields.
// -------------------------------------------------------------------------
template <int PF, bool EXT, bool IMGU, bool FS>
__global__ __launch_bounds__(256) void k_reverse(StepArgs a) {
  constexpr int W = 9 + PF;
  constexpr int R = PF + 1;
  static_assert(W % R == 0, "prefetch distance must make the rings commensurate");
  __shared__ float ldsU_all[kWavesPerBlock][kWave + 2 * kRadius];
  __shared__ float ldsL_all[kWavesPerBlock][kWave + 2 * kRadius];
  const int lane = threadIdx.x & 63;
  const int wv = uniform(threadIdx.x >> 6);
  int slot, tile;
  if (!map_tile(a.d, a.S, a.xcd_map, wv, slot, tile)) return;
  if (*a.err) return;
  const SlotInfo si = a.slots[slot];
  if (si.shot < 0) return;
  const ShotDesc sd = a.shots[si.shot];
  const int m = sd.nt - 1 - step_of(a);
  if (m < 1) return;

  const Dims& d = a.d;
  float* ldsU = ldsU_all[wv];
  float* ldsL = ldsL_all[wv];
  const int xt = tile % d.XT, zt = tile / d.XT;
  const int xs0 = xt * kWave;
  const Col col = make_col(d, xs0, lane);
  const int hmx = col.hcol - d.mx0;
  const bool hmcol = hmx >= 0 && hmx < d.nx;
  const int z0 = (FS ? d.ztop : 0) + zt * d.TZ, z1 = min(z0 + d.TZ, d.Z);
  float* ubase = a.u + (int64_t)si.cs * a.ustride;
  float* u_m = ubase + (int64_t)(m & 1) * d.field;  // u[m] in, u[m-2] out
  const float* u_m1 = ubase + (int64_t)((m - 1) & 1) * d.field;
  float* lbase = a.lam + (int64_t)slot * a.lstride;
  const float* l_p1 = lbase + (int64_t)((m + 1) & 1) * d.field;  // lam[m+1]
  float* l_p2 = lbase + (int64_t)(m & 1) * d.field;              // lam[m+2] in, lam[m] out

  // snapshot reset: at m == a_k the model cells of u[m] and u[m-1] come from
  // snapshot k, and at m == a_k - 1 u[m] comes from it again, so that both
  // levels of the recursion restart from forward values (a reconstructed
  // level paired with an exact one would act as a velocity kick that grows)
  const int rem = sd.nt - 1 - m;
  const bool reset = rem > 0 && (rem % sd.K) == 0 && rem / sd.K <= sd.nsnap;
  const bool reset_prev = rem > 1 && ((rem - 1) % sd.K) == 0 && (rem - 1) / sd.K <= sd.nsnap;
  const float* ckpt = a.snap + (int64_t)si.cs * a.snap_stride;
  const float* snap0 = reset ? ckpt + (int64_t)(rem / sd.K - 1) * 2 * d.model : nullptr;
  const float* snap1 = reset ? snap0 + d.model : nullptr;
  const float* snapp = reset_prev ? ckpt + (int64_t)((rem - 1) / sd.K - 1) * 2 * d.model + d.model : nullptr;
  const float* u0src = reset ? snap0 : snapp;  // model-cell source of u[m] (null: u_m)
  const float* strip = (m >= 3) ? a.strip + (int64_t)si.cs * a.strip_stride + (int64_t)(m - 2) * d.ring
                                : nullptr;
  const bool first = (m == sd.nt - 1);
  const int ext_slot = EXT ? step_of(a) % a.ext_T : 0;
  float* G = a.g + (int64_t)slot * d.model;
  float* E = a.E + (int64_t)slot * d.model;

  const bool src_tile = sd.src_z >= z0 && sd.src_z < z1 && sd.src_xs >= xs0 && sd.src_xs < xs0 + kWave;
  const float fsrc = src_tile ? a.wavelet[(int64_t)si.shot * a.wstride + (m - 1)] : 0.0f;

  // tiles of even zt sweep down (increasing z), odd ones up: two vertically
  // neighbouring tiles then read the rows they share at about the same time
  // (the second read comes from L2)
  const int dz = (zt & 1) ? -1 : 1;
  const int zS = dz > 0 ? z0 : z1 - 1, nT = z1 - z0;
  int rp, rbeg, rend;
  {
    const RmapDir dir = a.rdir[sd.rdir + xt];
    rbeg = dir.begin;
    rend = dir.begin + dir.count;
    if (dz > 0) {
      rp = rbeg;
      while (rp < rend && a.rrows[rp].z < z0) ++rp;
    } else {
      rp = rend - 1;
      while (rp >= rbeg && a.rrows[rp].z >= z1) --rp;
    }
  }
  int rz = (rp >= rbeg && rp < rend) ? a.rrows[rp].z : INT_MAX;
  const float* psi = a.traces + (int64_t)m * a.ntrace;

  float uc[W], uh[W], lc[W], lh[W];
  float p0[R], pl[R], pw[R], pg[R], pe[R];
  // Every row issues the same loads and no loaded value goes through a
  // select, so the compiler waits only for the rows consumed now, never for
  // the prefetch: rows and halo columns just outside the grid read the zero
  // guard rows and columns of the layout; u outside the model rows +-4 is
  // loaded as it is (the forward's sponge values) and never used, since only
  // model rows take the Laplacian of u; model-grid indices are clamped.
  auto load_rows = [&](int r, float& cu, float& hu, float& cl, float& hl) {
    const int64_t ro = (int64_t)r * d.P;
    const bool mrow = reset && r >= d.N && r < d.N + d.nz;
    const int64_t mo = (int64_t)min(max(r - d.N, 0), d.nz - 1) * d.nx;
    cl = l_p1[ro + col.xs];
    hl = l_p1[ro + col.hsafe];
    cu = *((mrow && col.mcol) ? snap1 + mo + col.mx : u_m1 + ro + col.xs);
    hu = *((mrow && hmcol) ? snap1 + mo + hmx : u_m1 + ro + col.hsafe);
  };
  // operands of the update of row r (model-cell values only used there)
  auto load_pt = [&](int r, float& u0, float& l2, float& w, float& g, float& e) {
    const int rc = clamp_row(d, r);
    const int64_t idx = (int64_t)rc * d.P + col.xs;
    const int64_t mi = (int64_t)min(max(rc - d.N, 0), d.nz - 1) * d.nx + col.mxc;
    l2 = l_p2[idx];
    w = a.w[idx];
    u0 = *(u0src ? u0src + mi : u_m + idx);
    g = G[mi];
    e = E[mi];  // replaced by 0 on the first step where it is used
  };
  // only the first window of the top tile reaches above the model (free
  // surface: odd image); elsewhere the loads go out back to back
  if (FS && z0 == d.ztop) {
#pragma unroll
    for (int j = 0; j < 8 + PF; ++j) {
      float sg;
      load_rows(image_row(d, z0 - 4 + j, sg), uc[j], uh[j], lc[j], lh[j]);
      uc[j] *= sg;
      uh[j] *= sg;
      lc[j] *= sg;
      lh[j] *= sg;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8 + PF; ++j) load_rows(zS + dz * (j - 4), uc[j], uh[j], lc[j], lh[j]);
  }
#pragma unroll
  for (int j = 0; j < PF; ++j) load_pt(zS + dz * j, p0[j], pl[j], pw[j], pg[j], pe[j]);

  // sweep position j is row zS + dz j; the rings hold positions, and the
  // stencil is symmetric in z
  for (int jb = 0; jb < nT; jb += W) {
#pragma unroll
    for (int r = 0; r < W; ++r) {
      const int j = jb + r;
      if (j >= nT) break;
      const int z = zS + dz * j;
      {
        const int s = (r + 8 + PF) % W, q = (r + PF) % R;
        load_rows(z + dz * (4 + PF), uc[s], uh[s], lc[s], lh[s]);
        load_pt(z + dz * PF, p0[q], pl[q], pw[q], pg[q], pe[q]);
      }
      const int ctr = (r + 4) % W;
      const float cu = uc[ctr], cl = lc[ctr];
      lds_put(ldsU, lane, cu, uh[ctr]);
      lds_put(ldsL, lane, cl, lh[ctr]);
      wave_lds_fence();
      const Row row = make_row(d, z);
      float lapL = laplace<W>(lc, r + 4, ldsL, lane);
      const float lapU0 = row.model ? laplace<W>(uc, r + 4, ldsU, lane) : 0.0f;
      wave_lds_fence();
      // receiver row (rare): the adjoint source is read and waited for here
      if (z == rz) {
        const int tr = a.rmaps[a.rrows[rp].map + lane];
        if (tr >= 0) lapL += psi[tr];
        rp += dz;
        rz = (rp >= rbeg && rp < rend) ? a.rrows[rp].z : INT_MAX;
      }
      float lapU = lapU0;
      if (src_tile && z == sd.src_z && col.xs == sd.src_xs) lapU += fsrc;

      if (col.xin) {
        const int q = r % R;
        const int64_t idx = (int64_t)z * d.P + col.xs;
        const float wv_ = pw[q];
        const int dd = max(row.dz, col.dxs);
        const float lout =
            dd == 0 ? fmaf(wv_, lapL, 2.0f * cl - pl[q]) : sponge_update(a.sp_a, dd, cl, pl[q], wv_, lapL);
        l_p2[idx] = lout;
        if (dd == 0) {
          const int64_t mi = (int64_t)row.mz * d.nx + col.mx;
          const float D = wv_ * lapU;
          u_m[idx] = fmaf(wv_, lapU, 2.0f * cu - p0[q]);
          G[mi] = fmaf(lout, IMGU ? cu : D, pg[q]);
          E[mi] = fmaf(D, D, first ? 0.0f : pe[q]);
          if (EXT) {
            const int64_t xo = ((int64_t)slot * a.ext_T + ext_slot) * d.model + mi;
            a.ext_lam[xo] = lout;
            a.ext_D[xo] = D;
          }
        } else {
          const int ri = strip_index(row, col);
          if (ri >= 0) u_m[idx] = strip ? strip[ri] : 0.0f;
        }
      }
    }
  }
}

// -------------------------------------------------------------------------
// Two reverse steps per launch, A = step m and B = step m-1 (temporal
// blocking: the four field levels are read once and written once for two
// steps, and g, E are updated once).  A workgroup's 4 wavefronts compute step
// A on 256 adjacent columns and step B on the 248 inside them, so B's
// horizontal neighbours are A's own results; the rows of A's inputs and of
// A's results are exchanged through the workgroup's LDS (one barrier per
// row), and only the outer wavefronts load halo columns.  Along z, A runs 4
// rows ahead of B and over 4 more rows on either side of the band; A's
// results of the last 10 rows stay in register rings for B's vertical
// stencil, beside A's input window, which also holds B's point-wise operands
// u[m-1], lam[m+1].  The sweep reads one pair of u and lam levels and writes
// the other pair (alternating from launch to launch), because neighbouring
// workgroups read the inputs in their overlap.  Snapshot restarts fall on A
// (even snapshot spacing); the launch before a restart stores the snapshot's
// u[a_k], u[a_k - 1] into the model cells of the levels it writes, so no
// launch reads snapshots.  Launch q runs A at m = nt-1-2q; B is skipped when
// m = 1.
// A row whose update is the plain interior FMA on every lane of a wavefront
// (a model row of columns inside the model, without receiver or source)
// takes a branch-free path; the other rows the general one (sponge in FP64,
// strip ring, zero boundary, receivers, source).
// -------------------------------------------------------------------------
// Buffer-resource addressing: a uniform base (4 SGPRs), a per-lane 32-bit
// byte offset fixed for the whole sweep and a uniform 32-bit byte offset per
// row, so that a load costs no per-lane address arithmetic.  The resource
// covers the array; every offset used here stays inside it.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kCachePolicyNT = 2;  // the nt bit of a gfx950 buffer access's cache policy
__device__ __forceinline__ rsrc_t make_rsrc(const float* base, int64_t floats) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)(floats * 4), 0x00020000);
}
__device__ __forceinline__ float bld(rsrc_t r, uint32_t voff, int32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, 0));
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t voff, int32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, soff, 0);
}
// the same with the non-temporal hint (nt), for results that no later access
// of the launch reads, so that they do not displace the input lines that the
// launch's neighbouring bands and workgroups still read from L2 (the reverse
// sweep's wavefield stores: its launch time fell 1.8 % at 2048x768 and 3.3 %
// at 1024x384; with the hint on its g and E stores as well 0.4 % less, on
// the forward sweep's stores 4.7 % slower, on loads slower in every case)
__device__ __forceinline__ void bst_nt(rsrc_t r, uint32_t voff, int32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, soff, kCachePolicyNT);
}


// Two-step sweeps: the grid's last column block may own fewer than 248
// columns.  Its workgroup lanes at or past (owned columns + 8) feed nothing
// it stores (B's owned lanes read A's results up to 4 lanes further, A reads
// its inputs up to 4 more), so a wavefront made only of such lanes ends
// before the sweep; the per-row barrier then synchronises the others only
// (a workgroup barrier counts the wavefronts that have not ended).
__device__ __forceinline__ bool idle_wave(const Dims& d, int xs0, int wv) {
  const int blk0 = xs0 - kWave * wv;  // storage column of the workgroup's lane 0
  const int owned_end = min(kWavesPerBlock * kWave - kRadius, d.off + d.X - blk0);
  return kWave * wv >= owned_end + 2 * kRadius;
}

// (at least 4 wavefronts per SIMD: the compiler keeps the deeper prefetch
// within 128 VGPRs)
template <int PF, bool EXT>
__global__ __launch_bounds__(256, 4) void k_reverse2(StepArgs a) {
  // PF: rows of loads in flight ahead of A (1 or 3)
  constexpr int W = PF == 1 ? 10 : 12;  // register rings: the unrolled period
  constexpr int R = PF + 1;             // point-wise rings
  static_assert(W >= 9 + PF && W % R == 0, "ring lengths must fit the window and the unrolled period");
  constexpr int LR = kWavesPerBlock * kWave + 2 * kRadius;
  constexpr int CB = 2 * kRadius;  // column bias of the lane offsets (halo columns reach -4)
  // the workgroup's rows of A's inputs (u, lam) and of A's results (for B),
  // 256 columns plus the 4-column halos; rows alternate between two buffer
  // sets, so that one barrier per row suffices
  __shared__ float xrow[2][4][LR];
  const int lane = threadIdx.x & 63;
  const int wv = uniform(threadIdx.x >> 6);
  int slot, tile;
  if (!map_tile(a.d, a.S, a.xcd_map, wv, slot, tile)) return;
  if (*a.err) return;
  const SlotInfo si = a.slots[slot];
  if (si.shot < 0) return;
  const ShotDesc sd = a.shots[si.shot];
  const int q = step_of(a);
  const int m = sd.nt - 1 - 2 * q;  // step A
  if (m < 1) return;
  const bool hasB = m >= 2;

  const Dims& d = a.d;
  const int xt = tile % d.XT, zt = tile / d.XT;  // xt % 4 == wv: the workgroup's columns
  // lane 0's storage column; B owns the workgroup's columns 4 .. 251
  const int xs0 = tile2_x0(d.off, xt);
  if (idle_wave(d, xs0, wv)) return;
  Col col = make_col(d, xs0, lane);
  const bool own_col = (wv > 0 || lane >= kRadius) && (wv < kWavesPerBlock - 1 || lane < kWave - kRadius) && col.xin;
  // only the outer wavefronts load halo columns (wave 0 lanes 0..3 the left,
  // the last wave lanes 4..7 the right one)
  const bool hl_lane = (wv == 0 && lane < 4) || (wv == kWavesPerBlock - 1 && lane >= 4 && lane < 8);
  // lanes without a halo column load lane 0's (wave 0 and the inner ones) or
  // lane 4's (last wave) halo address, one line per wavefront; their value is
  // overwritten by the lane's own column in the LDS row
  col.hsafe = hl_lane ? col.hcol : (wv == kWavesPerBlock - 1 ? xs0 + kWave : xs0 - kRadius);
  const int cidx = kRadius + kWave * wv + lane;  // this lane's slot in the workgroup rows
  const int hidx = hl_lane ? (lane < 4 ? lane : kWavesPerBlock * kWave + lane) : cidx;
  const int z0 = zt * d.TZ, z1 = min(z0 + d.TZ, d.Z);  // B's (owned) rows
  const int za0 = z0 - kRadius, za1 = z1 + kRadius;    // A's rows
  const int mz_lo = d.N, mz_hi = d.N + d.nz;           // model rows
  const bool tile_int = xs0 >= d.mx0 && xs0 + kWave <= d.mx0 + d.nx;  // every lane a model column
  // the tile reaches the strip ring around the model (its columns or its rows)
  const bool ring_cols = (xs0 < d.mx0 && xs0 + kWave > d.mx0 - kRadius) ||
                         (xs0 < d.mx0 + d.nx + kRadius && xs0 + kWave > d.mx0 + d.nx);
  const bool ring_rows = (za0 < mz_lo && za1 > mz_lo - kRadius) || (za0 < mz_hi + kRadius && za1 > mz_hi);
  const bool ring = ring_cols || ring_rows;

  // level pairs: launches with even q read the pair the forward sweep left
  // (u[k] at level k & 1) and write levels 3, 4; odd q the other way round
  const bool even = (q & 1) == 0;
  const int uA0 = even ? (m & 1) : 3;        // u[m]
  const int uA1 = even ? ((m - 1) & 1) : 4;  // u[m-1]
  const int uO0 = even ? 3 : (m & 1);        // u[m-2]
  const int uO1 = even ? 4 : ((m - 1) & 1);  // u[m-3]
  const int lA1 = even ? ((m + 1) & 1) : 3;  // lam[m+1]
  const int lA2 = even ? (m & 1) : 2;        // lam[m+2]
  const int lO0 = even ? 2 : (m & 1);        // lam[m]
  const int lO1 = even ? 3 : ((m + 1) & 1);  // lam[m-1]
  float* ubase = a.u + (int64_t)si.cs * a.ustride;
  float* lbase = a.lam + (int64_t)slot * a.lstride;
  float* G = a.g + (int64_t)slot * d.model;
  float* E = a.E + (int64_t)slot * d.model;
  // extended imaging: lam and D of both steps (reverse steps 2q, 2q+1) into
  // the slot's ring of ext_T steps
  float* xlA = EXT ? a.ext_lam + ((int64_t)slot * a.ext_T + (2 * q) % a.ext_T) * d.model : nullptr;
  float* xdA = EXT ? a.ext_D + ((int64_t)slot * a.ext_T + (2 * q) % a.ext_T) * d.model : nullptr;
  float* xlB = EXT ? a.ext_lam + ((int64_t)slot * a.ext_T + (2 * q + 1) % a.ext_T) * d.model : nullptr;
  float* xdB = EXT ? a.ext_D + ((int64_t)slot * a.ext_T + (2 * q + 1) % a.ext_T) * d.model : nullptr;
  const float* strip_base = a.strip + (int64_t)si.cs * a.strip_stride;
  // resources: this slot's u levels and lam levels with the guard rows in
  // front, w, g and E of the slot (E at a fixed offset after g), the strips
  const rsrc_t rU = make_rsrc(ubase - d.guard, d.guard + a.ustride);
  const rsrc_t rL = make_rsrc(lbase - d.guard, d.guard + a.lstride);
  const rsrc_t rW = make_rsrc(a.w - CB, d.field + CB);
  const rsrc_t rG = make_rsrc(G, (E - G) + d.model);
  const rsrc_t rS = make_rsrc(strip_base, a.strip_stride);
  // byte offset of row 0 of a level within rU / rL, less the column bias
  auto lev = [&](int k) { return (int32_t)((d.guard + (int64_t)k * d.field - CB) * 4); };
  const int32_t ouA0 = lev(uA0), ouA1 = lev(uA1), ouO0 = lev(uO0), ouO1 = lev(uO1);
  const int32_t olA1 = lev(lA1), olA2 = lev(lA2), olO0 = lev(lO0), olO1 = lev(lO1);
  const int32_t oE = (int32_t)((E - G) * 4);
  const int32_t P4 = d.P * 4;

  const bool hasSA = m >= 3, hasSB = m >= 4;  // strips of u[m-2], u[m-3] exist
  const int32_t osA = hasSA ? (int32_t)((int64_t)(m - 2) * d.ring * 4) : 0;
  const int32_t osB = hasSB ? (int32_t)((int64_t)(m - 3) * d.ring * 4) : 0;
  const bool first = (m == sd.nt - 1);

  const bool src_tile = sd.src_z >= za0 && sd.src_z < za1 && sd.src_xs >= xs0 && sd.src_xs < xs0 + kWave;
  const int src_row = src_tile ? sd.src_z : INT_MIN;
  const float fA = src_tile ? a.wavelet[(int64_t)si.shot * a.wstride + (m - 1)] : 0.0f;
  const float fB = (src_tile && hasB) ? a.wavelet[(int64_t)si.shot * a.wstride + (m - 2)] : 0.0f;

  // Bands of even zt sweep down (increasing z), odd ones up, so that two
  // neighbouring bands read the rows they share at about the same time (the
  // second read then comes from L2).  A visits its rows in sweep order, B
  // follows 4 rows behind.
  const int dz = (zt & 1) ? -1 : 1;
  const int zA0 = dz > 0 ? za0 : za1 - 1;  // A's first row
  const int nA = za1 - za0;

  // receiver rows of this tile (sorted by z), one cursor for each step, in
  // sweep order; INT_MAX once past the last
  int rpA, rpB, rbeg, rend;
  {
    const RmapDir dir = a.rdir[sd.rdir2 + xt];
    rbeg = dir.begin;
    rend = dir.begin + dir.count;
    if (dz > 0) {
      rpA = rbeg;
      while (rpA < rend && a.rrows[rpA].z < za0) ++rpA;
      rpB = rpA;
      while (rpB < rend && a.rrows[rpB].z < z0) ++rpB;
    } else {
      rpA = rend - 1;
      while (rpA >= rbeg && a.rrows[rpA].z >= za1) --rpA;
      rpB = rpA;
      while (rpB >= rbeg && a.rrows[rpB].z >= z1) --rpB;
    }
  }
  auto rz_at = [&](int rp) { return (rp >= rbeg && rp < rend) ? a.rrows[rp].z : INT_MAX; };
  int rzA = rz_at(rpA);
  int rzB = rz_at(rpB);
  const float* psiA = a.traces + (int64_t)m * a.ntrace;
  const float* psiB = a.traces + (int64_t)(m - 1) * a.ntrace;

  // per-lane byte offsets, fixed for the sweep
  const uint32_t oc = (uint32_t)(col.xs + CB) * 4u;     // centre column
  const uint32_t oh = (uint32_t)(col.hsafe + CB) * 4u;  // halo column (lanes 0..7)
  const uint32_t om = (uint32_t)col.mxc * 4u;           // model column (clamped)
  auto mrow4 = [&](int r) { return (int32_t)(min(max(r - d.N, 0), d.nz - 1) * d.nx * 4); };
  // strip ring index of (row r, this lane) as a byte offset, 0 if none
  auto strip_off = [&](int r) { return (uint32_t)max(strip_index(make_row(d, r), col), 0) * 4u; };

  // rings indexed by sweep position p at slot (p + 4) % W
  float uc[W], lc[W];         // A's inputs u[m-1], lam[m+1]: positions j-4 .. j+5
  float uo[W], lo[W], dA[W];  // A's results u[m-2], lam[m], D of step m: positions j-9 .. j
  float wr[W];  // w: positions j-4 .. j+PF (B uses A's loads 4 rows later)
  float uh[R], lh[R], p0[R], pl[R], sa[R];  // A's halo columns, point-wise operands, strip value
  float gB[R], eB[R], sb[R];                // B's point-wise operands, strip value
  // every row issues the same loads (strip values: every row of a tile at
  // the ring): stencil rows just outside the grid read the zero guard rows,
  // point-wise rows are clamped into the grid (rows past it are never used)
  auto load_win = [&](int r, float& cu, float& cl) {
    cu = bld(rU, oc, ouA1 + r * P4);
    cl = bld(rL, oc, olA1 + r * P4);
  };
  auto load_ptA = [&](int r, float& hu, float& hl, float& u0, float& l2, float& w, float& st) {
    hu = bld(rU, oh, ouA1 + r * P4);
    hl = bld(rL, oh, olA1 + r * P4);
    const int rc = clamp_row(d, r);
    u0 = bld(rU, oc, ouA0 + rc * P4);
    l2 = bld(rL, oc, olA2 + rc * P4);
    w = bld(rW, oc, rc * P4);
    if (ring) st = bld(rS, strip_off(rc), osA);
  };
  auto load_ptB = [&](int r, float& g, float& e, float& st) {
    const int rc = clamp_row(d, r);
    const int32_t mo = mrow4(rc);
    g = bld(rG, om, mo);
    e = bld(rG, om, mo + oE);
    if (ring) st = bld(rS, strip_off(rc), osB);
  };
  // sweep position j is row zA0 + dz j; the rings hold positions, and the
  // stencil is symmetric in z, so both directions share the code
#pragma unroll
  for (int j = 0; j < 8 + PF; ++j) load_win(zA0 + dz * (j - kRadius), uc[j], lc[j]);
#pragma unroll
  for (int j = 0; j < R; ++j) sa[j] = sb[j] = 0.0f;
#pragma unroll
  for (int j = 0; j < W; ++j) uo[j] = lo[j] = dA[j] = wr[j] = 0.0f;
#pragma unroll
  for (int j = 0; j < PF; ++j) {
    load_ptA(zA0 + dz * j, uh[j], lh[j], p0[j], pl[j], wr[(j + 4) % W], sa[j]);
    load_ptB(zA0 + dz * kRadius, gB[j], eB[j], sb[j]);  // (B's first row: B starts at position 8)
  }

  for (int jb = 0; jb < nA; jb += W) {
    static_for<W>([&](auto rc) __attribute__((always_inline)) {
      constexpr int r = decltype(rc)::value;
      const int j = jb + r;
      if (j >= nA) return;
      const int z = zA0 + dz * j;  // A's row; B's row is 4 rows behind
      load_win(z + dz * (kRadius + PF), uc[(r + 8 + PF) % W], lc[(r + 8 + PF) % W]);
      {
        const int qn = (r + PF) % R;
        load_ptA(z + dz * PF, uh[qn], lh[qn], p0[qn], pl[qn], wr[(r + 4 + PF) % W], sa[qn]);
        // B's operands PF positions ahead; before B starts, its first row
        // (the rows above it belong to the neighbouring band)
        load_ptB(zA0 + dz * (max(j + PF, 2 * kRadius) - kRadius), gB[qn], eB[qn], sb[qn]);
      }
      const int sA = (r + 4) % W;  // ring slot of row z
      const int sB = r % W;        // ring slot of row z - 4
      const int qa = r % R;
      // ---- the workgroup's rows: A's inputs at row z, A's results 4 rows behind
      float(*xr)[LR] = xrow[r & 1];
      xr[0][hidx] = uh[qa];
      xr[0][cidx] = uc[sA];
      xr[1][hidx] = lh[qa];
      xr[1][cidx] = lc[sA];
      xr[2][cidx] = uo[sB];
      xr[3][cidx] = lo[sB];
      // LDS-only release/acquire around the barrier: the loads in flight stay
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
      // ---- step A at row z (all 64 columns)
      float lapL = laplace<W>(lc, r + 4, xr[1] + kWave * wv, lane);
      float lapU = laplace<W>(uc, r + 4, xr[0] + kWave * wv, lane);
      {
        const float w = wr[sA], cu = uc[sA], cl = lc[sA];
        float lo_ = 0.0f, uo_ = 0.0f, d_ = 0.0f;
        if (tile_int && z >= mz_lo && z < mz_hi && z != rzA && z != src_row) {
          lo_ = fmaf(w, lapL, 2.0f * cl - pl[qa]);
          d_ = w * lapU;
          uo_ = fmaf(w, lapU, 2.0f * cu - p0[qa]);
        } else if (z >= 0 && z < d.Z) {
          if (z == rzA) {
            const int tr = a.rmaps[a.rrows[rpA].map + lane];
            if (tr >= 0) lapL += psiA[tr];
            rpA += dz;
            rzA = rz_at(rpA);
          }
          if (z == src_row && col.xs == sd.src_xs) lapU += fA;
          const Row row = make_row(d, z);
          const int dd = max(row.dz, col.dxs);
          if (col.xin && dd == 0) {
            lo_ = fmaf(w, lapL, 2.0f * cl - pl[qa]);
            d_ = w * lapU;
            uo_ = fmaf(w, lapU, 2.0f * cu - p0[qa]);
          } else if (col.xin) {
            lo_ = sponge_update(a.sp_a, dd, cl, pl[qa], w, lapL);
            if (hasSA && strip_index(row, col) >= 0) uo_ = sa[qa];
          }
        }
        if (z >= z0 && z < z1 && own_col) {
          bst_nt(rU, oc, ouO0 + z * P4, uo_);
          bst_nt(rL, oc, olO0 + z * P4, lo_);
          if (EXT && z >= mz_lo && z < mz_hi && col.mcol) {
            const int64_t mi = (int64_t)(z - d.N) * d.nx + col.mx;
            xlA[mi] = lo_;
            xdA[mi] = d_;
          }
        }
        uo[sA] = uo_;
        lo[sA] = lo_;
        dA[sA] = d_;
      }
      // ---- step B at row z - 4 dz (owned lanes), from sweep position 8 on
      const int zbB = z - dz * kRadius;
      if (j >= 2 * kRadius) {
        const int qb = r % R;
        float lapLB = laplace<W>(lo, r, xr[3] + kWave * wv, lane);
        float lapUB = laplace<W>(uo, r, xr[2] + kWave * wv, lane);
        const float w = wr[sB], cu = uo[sB], cl = lo[sB], pu = uc[sB], pl1 = lc[sB], da = dA[sB];
        float l1 = 0.0f, u1 = 0.0f, gn = 0.0f, en = 0.0f, dB = 0.0f;
        bool st_l = own_col, st_u = own_col, st_g = own_col;
        if (tile_int && zbB >= mz_lo && zbB < mz_hi && zbB != rzB && zbB != src_row && hasB) {
          l1 = fmaf(w, lapLB, 2.0f * cl - pl1);
          const float D = w * lapUB;
          dB = D;
          u1 = fmaf(w, lapUB, 2.0f * cu - pu);
          gn = fmaf(l1, D, fmaf(cl, da, gB[qb]));
          en = fmaf(D, D, fmaf(da, da, first ? 0.0f : eB[qb]));
        } else {
          if (zbB == rzB) {
            const int tr = a.rmaps[a.rrows[rpB].map + lane];
            if (tr >= 0 && hasB) lapLB += psiB[tr];
            rpB += dz;
            rzB = rz_at(rpB);
          }
          if (zbB == src_row && col.xs == sd.src_xs) lapUB += fB;
          const Row row = make_row(d, zbB);
          const int dd = max(row.dz, col.dxs);
          st_l = own_col && hasB;
          st_g = own_col && dd == 0;
          if (dd == 0) {
            const float ag = fmaf(cl, da, gB[qb]);
            const float ae = fmaf(da, da, first ? 0.0f : eB[qb]);
            l1 = fmaf(w, lapLB, 2.0f * cl - pl1);
            const float D = w * lapUB;
            dB = D;
            u1 = fmaf(w, lapUB, 2.0f * cu - pu);
            gn = hasB ? fmaf(l1, D, ag) : ag;
            en = hasB ? fmaf(D, D, ae) : ae;
            st_u = st_l;
          } else {
            l1 = sponge_update(a.sp_a, dd, cl, pl1, w, lapLB);
            u1 = hasSB ? sb[qb] : 0.0f;
            st_u = st_l && strip_index(row, col) >= 0;
          }
        }
        if (st_l) bst_nt(rL, oc, olO1 + zbB * P4, l1);
        if (st_u) bst_nt(rU, oc, ouO1 + zbB * P4, u1);
        if (st_g) {
          const int32_t mo = mrow4(zbB);
          bst(rG, om, mo, gn);
          bst(rG, om, mo + oE, en);
          if (EXT && hasB) {  // (st_g: a model cell of this wavefront)
            const int64_t mi = (int64_t)(zbB - d.N) * d.nx + col.mx;
            xlB[mi] = l1;
            xdB[mi] = dB;
          }
        }
      }
    });
  }

  // the next launch restarts from snapshot k: its inputs u[m-2], u[m-3] take
  // the snapshot's values in the model cells (after this wavefront's own
  // stores of the reconstructed values, which only this launch used)
  const int remn = sd.nt - 1 - (m - 2);
  if (m - 2 >= 1 && (remn % sd.K) == 0 && remn / sd.K <= sd.nsnap) {
    const float* sn0 = a.snap + (int64_t)si.cs * a.snap_stride + (int64_t)(remn / sd.K - 1) * 2 * d.model;
    const float* sn1 = sn0 + d.model;
    float* u0 = ubase + (int64_t)uO0 * d.field;
    float* u1 = ubase + (int64_t)uO1 * d.field;
    if (own_col && col.mcol) {
      for (int z = max(z0, mz_lo); z < min(z1, mz_hi); ++z) {
        const int64_t mi = (int64_t)(z - d.N) * d.nx + col.mx;
        const int64_t idx = (int64_t)z * d.P + col.xs;
        u0[idx] = sn0[mi];
        u1[idx] = sn1[mi];
      }
    }
  }
}

// -------------------------------------------------------------------------
// Two forward steps per launch for the gradient's forward sweep (recording,
// checkpoints; no free surface), A = step n -> n+1 and B = step n+1 -> n+2,
// with the workgroup tiling of the two-step reverse sweep: A on 256 columns,
// B on the 248 inside them, rows exchanged through LDS with one barrier per
// row, A 4 rows ahead of B and over 4 more rows on either side of the band,
// A's results u[n+1], d[n+1] of the last 10 (12) rows in register rings.
// The u levels hold two sets of (u[k] at k & 1, d) in levels 0-2 and 3-5: a
// launch reads one set and writes u[n+1], u[n+2], d[n+2] into the other
// (neighbouring workgroups read the inputs in their overlap); u[n+1] only in
// a shot's last launch.  A shot whose last launch ends after A (an odd
// number of steps) stores u[n], u[n+1], d[n+1] instead.  Strips, snapshots and traces are written by the step
// that produces them, as in the one-step sweep.
// -------------------------------------------------------------------------
template <int PF>
__global__ __launch_bounds__(256, 4) void k_forward2(StepArgs a) {
  constexpr int W = PF == 1 ? 10 : 12;  // register rings: the unrolled period
  constexpr int R = PF + 1;             // point-wise rings
  static_assert(W >= 9 + PF && W % R == 0, "ring lengths must fit the window and the unrolled period");
  constexpr int LR = kWavesPerBlock * kWave + 2 * kRadius;
  constexpr int CB = 2 * kRadius;  // column bias of the lane offsets
  // the workgroup's rows of A's input u[n] (with the halos) and of A's result
  // u[n+1] (for B); rows alternate between two buffer sets
  __shared__ float xrow[2][2][LR];
  const int lane = threadIdx.x & 63;
  const int wv = uniform(threadIdx.x >> 6);
  int slot, tile;
  if (!map_tile(a.d, a.S, a.xcd_map, wv, slot, tile)) return;
  if (*a.err) return;
  const SlotInfo si = a.slots[slot];
  if (si.shot < 0) return;
  const ShotDesc sd = a.shots[si.shot];
  const int q = step_of(a);
  const int n = 2 * q;  // step A: n -> n+1
  if (n >= sd.nt - 1) return;
  const bool hasB = n + 1 < sd.nt - 1;
  // u[n+1] is stored only by the shot's last launch (the reverse sweep starts
  // from u[nt-1], u[nt-2]); the next launch reads u[n+2] and d[n+2] only
  const bool keep1 = n + 2 >= sd.nt - 1;

  const Dims& d = a.d;
  const int xt = tile % d.XT, zt = tile / d.XT;  // xt % 4 == wv
  const int xs0 = tile2_x0(d.off, xt);
  if (idle_wave(d, xs0, wv)) return;
  Col col = make_col(d, xs0, lane);
  const bool own_col = (wv > 0 || lane >= kRadius) && (wv < kWavesPerBlock - 1 || lane < kWave - kRadius) && col.xin;
  const bool hl_lane = (wv == 0 && lane < 4) || (wv == kWavesPerBlock - 1 && lane >= 4 && lane < 8);
  // lanes without a halo column load lane 0's (wave 0 and the inner ones) or
  // lane 4's (last wave) halo address, one line per wavefront; their value is
  // overwritten by the lane's own column in the LDS row
  col.hsafe = hl_lane ? col.hcol : (wv == kWavesPerBlock - 1 ? xs0 + kWave : xs0 - kRadius);
  const int cidx = kRadius + kWave * wv + lane;
  const int hidx = hl_lane ? (lane < 4 ? lane : kWavesPerBlock * kWave + lane) : cidx;
  const int z0 = zt * d.TZ, z1 = min(z0 + d.TZ, d.Z);  // B's (owned) rows
  const int za0 = z0 - kRadius, za1 = z1 + kRadius;    // A's rows
  const int mz_lo = d.N, mz_hi = d.N + d.nz;
  const bool tile_int = xs0 >= d.mx0 && xs0 + kWave <= d.mx0 + d.nx;

  // level sets: launch q reads set q & 1 and writes the other
  const int si_ = 3 * (q & 1), so_ = 3 - si_;
  const int uIn = si_ + (n & 1), dIn = si_ + 2;
  const int uO1 = so_ + ((n + 1) & 1), uO0 = so_ + (n & 1), dO = so_ + 2;  // u[n+1]; u[n+2] (or u[n]); d
  float* ubase = a.u + (int64_t)si.cs * a.ustride;
  const rsrc_t rU = make_rsrc(ubase - d.guard, d.guard + a.ustride);
  const rsrc_t rW = make_rsrc(a.w - CB, d.field + CB);
  auto lev = [&](int k) { return (int32_t)((d.guard + (int64_t)k * d.field - CB) * 4); };
  const int32_t ouIn = lev(uIn), odIn = lev(dIn), ouO1 = lev(uO1), ouO0 = lev(uO0), odO = lev(dO);
  const int32_t P4 = d.P * 4;

  // strips of u[n+1], u[n+2]; snapshot pairs saved at A or at B
  float* strip_base = a.strip + (int64_t)si.cs * a.strip_stride;
  float* stripA = strip_base + (int64_t)(n + 1) * d.ring;
  float* stripB = strip_base + (int64_t)(n + 2) * d.ring;
  const int remA = sd.nt - 2 - n, remB = remA - 1;
  const bool saveA = remA > 0 && (remA % sd.K) == 0;
  const bool saveB = hasB && remB > 0 && (remB % sd.K) == 0;
  float* ckpt = a.snap + (int64_t)si.cs * a.snap_stride;
  float* snA0 = saveA ? ckpt + (int64_t)(remA / sd.K - 1) * 2 * d.model : nullptr;
  float* snB0 = saveB ? ckpt + (int64_t)(remB / sd.K - 1) * 2 * d.model : nullptr;

  const bool src_tile = sd.src_z >= za0 && sd.src_z < za1 && sd.src_xs >= xs0 && sd.src_xs < xs0 + kWave;
  const int src_row = src_tile ? sd.src_z : INT_MIN;
  const float fA = src_tile ? a.wavelet[(int64_t)si.shot * a.wstride + n] : 0.0f;
  const float fB = (src_tile && hasB) ? a.wavelet[(int64_t)si.shot * a.wstride + n + 1] : 0.0f;

  // bands alternate direction (neighbours read their shared rows together)
  const int dz = (zt & 1) ? -1 : 1;
  const int zA0 = dz > 0 ? za0 : za1 - 1;
  const int nA = za1 - za0;
  int rpA, rpB, rbeg, rend;
  {
    const RmapDir dir = a.rdir[sd.rdir2 + xt];
    rbeg = dir.begin;
    rend = dir.begin + dir.count;
    if (dz > 0) {
      rpA = rbeg;
      while (rpA < rend && a.rrows[rpA].z < za0) ++rpA;
      rpB = rpA;
      while (rpB < rend && a.rrows[rpB].z < z0) ++rpB;
    } else {
      rpA = rend - 1;
      while (rpA >= rbeg && a.rrows[rpA].z >= za1) --rpA;
      rpB = rpA;
      while (rpB >= rbeg && a.rrows[rpB].z >= z1) --rpB;
    }
  }
  auto rz_at = [&](int rp) { return (rp >= rbeg && rp < rend) ? a.rrows[rp].z : INT_MAX; };
  int rzA = rz_at(rpA), rzB = rz_at(rpB);
  float* trA = a.traces + (int64_t)(n + 1) * a.ntrace;
  float* trB = a.traces + (int64_t)(n + 2) * a.ntrace;

  const uint32_t oc = (uint32_t)(col.xs + CB) * 4u;
  const uint32_t oh = (uint32_t)(col.hsafe + CB) * 4u;

  // rings indexed by sweep position p at slot (p + 4) % W
  float uc[W];          // A's input u[n]: positions j-4 .. j+5
  float uo[W], dq[W];   // A's results u[n+1], d[n+1]: positions j-9 .. j
  float wr[W];          // w: positions j-4 .. j+PF (B uses A's loads 4 rows later)
  float uh[R], pd[R];   // A's halo column, d[n]
  auto load_ptA = [&](int r, float& hu, float& dn, float& w) {
    hu = bld(rU, oh, ouIn + r * P4);
    const int rc = clamp_row(d, r);
    dn = bld(rU, oc, odIn + rc * P4);
    w = bld(rW, oc, rc * P4);
  };
#pragma unroll
  for (int j = 0; j < 8 + PF; ++j) uc[j] = bld(rU, oc, ouIn + (zA0 + dz * (j - kRadius)) * P4);
#pragma unroll
  for (int j = 0; j < W; ++j) wr[j] = 0.0f;
#pragma unroll
  for (int j = 0; j < PF; ++j) load_ptA(zA0 + dz * j, uh[j], pd[j], wr[(j + 4) % W]);
#pragma unroll
  for (int j = 0; j < W; ++j) uo[j] = dq[j] = 0.0f;

  for (int jb = 0; jb < nA; jb += W) {
    static_for<W>([&](auto rc) __attribute__((always_inline)) {
      constexpr int r = decltype(rc)::value;
      const int j = jb + r;
      if (j >= nA) return;
      const int z = zA0 + dz * j;  // A's row; B's row is 4 rows behind
      uc[(r + 8 + PF) % W] = bld(rU, oc, ouIn + (z + dz * (kRadius + PF)) * P4);
      {
        const int qn = (r + PF) % R;
        load_ptA(z + dz * PF, uh[qn], pd[qn], wr[(r + 4 + PF) % W]);
      }
      const int sA = (r + 4) % W, sB = r % W, qa = r % R;
      float(*xr)[LR] = xrow[r & 1];
      xr[0][hidx] = uh[qa];
      xr[0][cidx] = uc[sA];
      xr[1][cidx] = uo[sB];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
      // ---- step A at row z
      {
        float lap = laplace<W>(uc, r + 4, xr[0] + kWave * wv, lane);
        const float c = uc[sA], dn = pd[qa], w = wr[sA];
        float out = 0.0f, dnew = 0.0f;
        const bool own_row = z >= z0 && z < z1;
        if (tile_int && z >= mz_lo && z < mz_hi && z != rzA && z != src_row && !saveA) {
          dnew = fmaf(w, lap, dn);
          out = c + dnew;
        } else if (z >= 0 && z < d.Z) {
          if (z == src_row && col.xs == sd.src_xs) lap += fA;
          const Row row = make_row(d, z);
          if (col.xin) {
            const int dd = max(row.dz, col.dxs);
            if (dd == 0) {
              dnew = fmaf(w, lap, dn);
            } else {
              const double gm = a.sp_a * (double)(dd * dd);
              dnew = (float)(((1.0 - gm) * (double)dn + (double)w * (double)lap) / (1.0 + gm));
            }
            out = c + dnew;
            if (own_row && own_col) {
              const int ri = strip_index(row, col);
              if (ri >= 0) stripA[ri] = out;
              if (saveA && row.model && col.mcol) {
                const int64_t mi = (int64_t)row.mz * d.nx + col.mx;
                snA0[mi] = out;
                snA0[d.model + mi] = c;
              }
            }
          }
          if (z == rzA) {
            const int tr = a.rmaps[a.rrows[rpA].map + lane];
            if (tr >= 0 && own_col) trA[tr] = out;
            rpA += dz;
            rzA = rz_at(rpA);
          }
        }
        if (own_row && own_col) {
          if (keep1) bst(rU, oc, ouO1 + z * P4, out);
          if (!hasB) {
            bst(rU, oc, ouO0 + z * P4, c);
            bst(rU, oc, odO + z * P4, dnew);
          }
        }
        uo[sA] = out;
        dq[sA] = dnew;
      }
      // ---- step B at row z - 4 dz, from sweep position 8 on
      const int zbB = z - dz * kRadius;
      if (hasB && j >= 2 * kRadius) {
        float lap = laplace<W>(uo, r, xr[1] + kWave * wv, lane);
        const float c = uo[sB], dn = dq[sB], w = wr[sB];
        float out, dnew;
        if (tile_int && zbB >= mz_lo && zbB < mz_hi && zbB != rzB && zbB != src_row && !saveB) {
          dnew = fmaf(w, lap, dn);
          out = c + dnew;
        } else {
          if (zbB == src_row && col.xs == sd.src_xs) lap += fB;
          const Row row = make_row(d, zbB);
          const int dd = max(row.dz, col.dxs);
          if (dd == 0) {
            dnew = fmaf(w, lap, dn);
          } else {
            const double gm = a.sp_a * (double)(dd * dd);
            dnew = (float)(((1.0 - gm) * (double)dn + (double)w * (double)lap) / (1.0 + gm));
          }
          out = c + dnew;
          if (own_col) {
            const int ri = strip_index(row, col);
            if (ri >= 0) stripB[ri] = out;
            if (saveB && row.model && col.mcol) {
              const int64_t mi = (int64_t)row.mz * d.nx + col.mx;
              snB0[mi] = out;
              snB0[d.model + mi] = c;
            }
          }
          if (zbB == rzB) {
            const int tr = a.rmaps[a.rrows[rpB].map + lane];
            if (tr >= 0 && own_col) trB[tr] = out;
            rpB += dz;
            rzB = rz_at(rpB);
          }
        }
        if (own_col) {
          bst(rU, oc, ouO0 + zbB * P4, out);
          bst(rU, oc, odO + zbB * P4, dnew);
        }
      }
    });
  }
}

// -------------------------------------------------------------------------
// offset-extended imaging condition over a window of reverse steps:
//   I(x, h) += sum_slots sum_m lam[m](x - h) D[m](x + h),  |h| <= hmax <= HM
// One wavefront owns 64 model columns of one model row and keeps the 2HM+1
// offset sums in registers over all slots and steps of the window; each
// step's lam and D rows (with HM columns on each side, zero outside the
// model) are staged in the wavefront's LDS rows, and the sums are added to I
// once per window.
// -------------------------------------------------------------------------
template <int HM>
__global__ __launch_bounds__(256) void k_ext_image(ExtArgs a) {
  constexpr int L = kWave + 2 * HM;
  __shared__ float shL_all[kWavesPerBlock][L];
  __shared__ float shD_all[kWavesPerBlock][L];
  const Dims& d = a.d;
  const int lane = threadIdx.x & 63;
  const int wv = uniform(threadIdx.x >> 6);
  const int XTm = (d.nx + kWave - 1) / kWave;
  const int wave = blockIdx.x * kWavesPerBlock + wv;
  if (wave >= d.nz * XTm || *a.err) return;
  const int iz = wave / XTm, x0 = (wave % XTm) * kWave;
  const int x = x0 + lane;
  float* shL = shL_all[wv];
  float* shD = shD_all[wv];
  const int H = a.hmax;
  const int j0 = (a.step_ctr ? a.step_mul * *a.step_ctr : 0) + a.step0;
  float acc[2 * HM + 1];
#pragma unroll
  for (int h = 0; h < 2 * HM + 1; ++h) acc[h] = 0.0f;
  for (int s = 0; s < a.S; ++s) {
    const SlotInfo si = a.slots[s];
    if (si.shot < 0) continue;
    const int nt = a.shots[si.shot].nt;
    for (int k = 0; k < a.count; ++k) {
      const int j = j0 + k;
      if (nt - 1 - j < 1) break;  // this slot's shot is done from here on
      const int64_t row = ((int64_t)s * a.T + j % a.T) * d.model + (int64_t)iz * d.nx;
      for (int c = lane; c < L; c += kWave) {
        const int xx = x0 - HM + c;
        const bool in = xx >= 0 && xx < d.nx;
        shL[c] = in ? a.lam[row + xx] : 0.0f;
        shD[c] = in ? a.D[row + xx] : 0.0f;
      }
      wave_lds_fence();
#pragma unroll
      for (int h = -HM; h <= HM; ++h)
        if (h >= -H && h <= H) acc[h + HM] = fmaf(shL[lane + HM - h], shD[lane + HM + h], acc[h + HM]);
      wave_lds_fence();
    }
  }
  if (x >= d.nx) return;
  const int64_t cell = (int64_t)iz * d.nx + x;
#pragma unroll
  for (int h = -HM; h <= HM; ++h)
    if (h >= -H && h <= H) a.I[(int64_t)(h + H) * d.model + cell] += acc[h + HM];
}

// Four columns per lane: each lane keeps the 2HM+1 sums of 4 adjacent
// columns, reads its 4 + 2HM operands of lam and D per step as float4 rows
// from LDS (one read per operand serves up to four products instead of one),
// and the next step's rows are loaded while the current one is folded.  The
// slots are split into `groups` so that enough wavefronts run; each group
// adds into its own partial image.
template <int HM>
__global__ __launch_bounds__(256) void k_ext_image4(ExtArgs a) {
  constexpr int C = 4;
  constexpr int TW = kWave * C;           // columns per wavefront
  constexpr int L = TW + 2 * HM;          // staged row length
  constexpr int NL = (L + kWave - 1) / kWave;
  constexpr int WIN = C + 2 * HM;         // operands one lane reads
  static_assert(HM % 4 == 0, "window reads are float4");
  __shared__ __align__(16) float shL_all[kWavesPerBlock][L];
  __shared__ __align__(16) float shD_all[kWavesPerBlock][L];
  const Dims& d = a.d;
  const int lane = threadIdx.x & 63;
  const int wv = uniform(threadIdx.x >> 6);
  const int XTw = (d.nx + TW - 1) / TW;
  const int per_group = d.nz * XTw;
  const int wave = blockIdx.x * kWavesPerBlock + wv;
  if (wave >= per_group * a.groups || *a.err) return;
  const int grp = wave / per_group, rem = wave % per_group;
  const int iz = rem / XTw, x0 = (rem % XTw) * TW;
  const int spg = (a.S + a.groups - 1) / a.groups;
  const int s_lo = grp * spg, s_hi = min(a.S, s_lo + spg);
  const int H = a.hmax;
  const int j0 = (a.step_ctr ? a.step_mul * *a.step_ctr : 0) + a.step0;
  const int n_it = max(s_hi - s_lo, 0) * a.count;
  float* shL = shL_all[wv];
  float* shD = shD_all[wv];
  float acc[C][2 * HM + 1];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int h = 0; h < 2 * HM + 1; ++h) acc[c][h] = 0.0f;
  float nl[NL], nd[NL];
  // loads of iteration `it` = (slot s_lo + it / count, step it % count); a
  // slot whose shot has ended contributes zeros
  auto issue = [&](int it) {
    const int s = s_lo + it / a.count, j = j0 + it % a.count;
    const SlotInfo si = a.slots[s];
    const bool ok = si.shot >= 0 && a.shots[si.shot].nt - 1 - j >= 1;
    const int64_t row = ((int64_t)s * a.T + j % a.T) * d.model + (int64_t)iz * d.nx;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int c = lane + kWave * q;
      const int xx = x0 - HM + c;
      const bool in = ok && c < L && xx >= 0 && xx < d.nx;
      nl[q] = in ? a.lam[row + xx] : 0.0f;
      nd[q] = in ? a.D[row + xx] : 0.0f;
    }
  };
  if (n_it > 0) issue(0);
  for (int it = 0; it < n_it; ++it) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int c = lane + kWave * q;
      if (c < L) {
        shL[c] = nl[q];
        shD[c] = nd[q];
      }
    }
    if (it + 1 < n_it) issue(it + 1);
    wave_lds_fence();
    float lw[WIN], dw[WIN];
#pragma unroll
    for (int k = 0; k < WIN / 4; ++k) {
      const float4 tl = *reinterpret_cast<const float4*>(shL + C * lane + 4 * k);
      const float4 td = *reinterpret_cast<const float4*>(shD + C * lane + 4 * k);
      lw[4 * k] = tl.x; lw[4 * k + 1] = tl.y; lw[4 * k + 2] = tl.z; lw[4 * k + 3] = tl.w;
      dw[4 * k] = td.x; dw[4 * k + 1] = td.y; dw[4 * k + 2] = td.z; dw[4 * k + 3] = td.w;
    }
    // column x0 + C lane + c, offset h: lam at window index c + HM - h, D at c + HM + h
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int h = -HM; h <= HM; ++h)
        if (h >= -H && h <= H) acc[c][h + HM] = fmaf(lw[c + HM - h], dw[c + HM + h], acc[c][h + HM]);
    wave_lds_fence();
  }
  float* I = a.I + (int64_t)grp * (2 * H + 1) * d.model;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int x = x0 + C * lane + c;
    if (x >= d.nx) continue;
    const int64_t cell = (int64_t)iz * d.nx + x;
#pragma unroll
    for (int h = -HM; h <= HM; ++h)
      if (h >= -H && h <= H) I[(int64_t)(h + H) * d.model + cell] += acc[c][h + HM];
  }
}

// image(x, h) = (2 / v(x)^3) sum over groups of Iacc[g](x, h), fixed order
__global__ void k_ext_out(Dims d, const float* Iacc, int groups, int nh, const float* v, float* image,
                          const int32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.model * nh) return;
  const int64_t cell = i % d.model;
  double sum = 0.0;
  for (int g = 0; g < groups; ++g) sum += (double)Iacc[(int64_t)g * nh * d.model + i];
  const double vv = v[cell];
  image[i] = (*err) ? NAN : (float)(2.0 / (vv * vv * vv) * sum);
}

// -------------------------------------------------------------------------
// small kernels
// -------------------------------------------------------------------------
__global__ void k_prep(Dims d, const float* __restrict__ v, float* __restrict__ w, double dt2_h2,
                       float vmax, int32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.field) return;
  const int z = (int)(i / d.P), xs = (int)(i % d.P), x = xs - d.off;
  float out = 0.0f;
  if (x >= 0 && x < d.X && z < d.Z) {
    const int iz = min(max(z - d.N, 0), d.nz - 1), ix = min(max(x - d.N, 0), d.nx - 1);
    const float vv = v[(int64_t)iz * d.nx + ix];
    if (!(vv > 0.0f && vv <= vmax)) atomicOr(err, 1);
    out = (float)(dt2_h2 * (double)vv * (double)vv);
  }
  w[i] = out;
}

__global__ void k_prep_born(Dims d, const float* __restrict__ v, const float* __restrict__ dv,
                            float* __restrict__ bw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.field) return;
  const int z = (int)(i / d.P), xs = (int)(i % d.P);
  const int mz = z - d.N, mx = xs - d.mx0;
  float out = 0.0f;
  if (mz >= 0 && mz < d.nz && mx >= 0 && mx < d.nx) {
    const int64_t m = (int64_t)mz * d.nx + mx;
    out = 2.0f * dv[m] / v[m];
  }
  bw[i] = out;
}

__global__ void k_fill(uint32_t* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = i; k < n; k += stride) p[k] = 0u;
}

__global__ void k_fill_slots(float* base, int64_t stride, int64_t count, const SlotInfo* slots,
                             int use_cs) {
  const SlotInfo si = slots[blockIdx.y];
  if (si.shot < 0) return;
  float* p = base + (int64_t)(use_cs ? si.cs : (int)blockIdx.y) * stride;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    p[k] = 0.0f;
}

__global__ void k_advance(int32_t* ctr, int32_t by) { *ctr += by; }
__global__ void k_set(int32_t* ctr, int32_t value) { *ctr = value; }

// misfit of one trace per thread; psi' = psi * h^2/dt^2 written in place.
// kind 0: J and psi of the plain misfit; 1: of eq. (2); 2: J of eq. (2) with
// the plain-residual psi (for eq. (3) taken literally)
__global__ void k_misfit(MisfitArgs a) {
  const SlotInfo si = a.slots[blockIdx.y];
  if (si.shot < 0 || *a.err) return;
  const ShotDesc sd = a.shots[si.shot];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= sd.nrec) return;
  const int tr = sd.rec_begin + r;
  float* syn = a.traces + tr;
  // no recorded data (Gauss-Newton products): the residual is the synthetic itself
  const float* obs = a.dobs ? a.dobs + (int64_t)tr * a.nt_max : nullptr;
  const int64_t st = a.ntrace;
  const int nt = sd.nt;
  double J = 0.0;
  if (a.kind == 0) {
    for (int t = 0; t < nt; ++t) {
      const double rr = (t == 0 ? 0.0 : (double)syn[t * st]) - (obs ? (double)obs[t] : 0.0);
      J += rr * rr;
      syn[t * st] = (float)(rr * a.psi_scale);
    }
  } else {
    // eq. (2): R[n] = dt sum_{k<=n} r[k]; psi[n] = dt sum_{k>=n} R[k] = dt (S - sum_{k<n} R[k])
    double R = 0.0, S = 0.0;
    for (int t = 0; t < nt; ++t) {
      const double rr = (t == 0 ? 0.0 : (double)syn[t * st]) - (obs ? (double)obs[t] : 0.0);
      R += a.dt * rr;
      J += R * R;
      S += R;
    }
    double Rp = 0.0, Pn = 0.0;
    for (int t = 0; t < nt; ++t) {
      const double rr = (t == 0 ? 0.0 : (double)syn[t * st]) - (obs ? (double)obs[t] : 0.0);
      Rp += a.dt * rr;
      syn[t * st] = (float)((a.kind == 2 ? rr : a.dt * (S - Pn)) * a.psi_scale);
      Pn += Rp;
    }
  }
  a.Jpart[tr] = 0.5 * J;
}

// deterministic fixed-order sum of per-trace misfits
__global__ __launch_bounds__(1024) void k_reduce_J(const double* part, int n, double* J,
                                                   const int32_t* err) {
  __shared__ double sh[1024];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *J = (*err) ? NAN : sh[0];
}

// per-batch Hessian epilogue over model rows: H1 += E_s/dt^3 and
// D(x,h) += (4/v^6) E_s(x+h)/dt^3 A_s(x-h).  A_s and E_s of each shot are
// staged in LDS for the tile plus HM cells on each side, so every asinh pair
// is evaluated once per cell and shot; HM is the compile-time offset bound.
constexpr int kEpiTile = 256;
template <int HM>
__global__ __launch_bounds__(kEpiTile) void k_epilogue(EpiArgs a) {
  __shared__ float shE[kEpiTile + 2 * HM];
  __shared__ float shA[kEpiTile + 2 * HM];
  const Dims& d = a.d;
  const int iz = blockIdx.y;
  const int x0 = blockIdx.x * kEpiTile;
  const int ix = x0 + threadIdx.x;
  const bool in = ix < d.nx;
  const int H = a.hmax;
  const int64_t cell = (int64_t)iz * d.nx + ix;
  float h1 = 0.0f;
  float acc[2 * HM + 1];
#pragma unroll
  for (int h = 0; h < 2 * HM + 1; ++h) acc[h] = 0.0f;
  const bool bad = *a.err != 0;
  for (int s = 0; s < a.S && !bad; ++s) {
    const SlotInfo si = a.slots[s];
    if (si.shot < 0) continue;
    const float* Es = a.E + (int64_t)s * d.model + (int64_t)iz * d.nx;
    if (a.H1 && in) h1 += Es[ix] * a.inv_dt3;
    if (!a.D) continue;
    const ShotDesc sd = a.shots[si.shot];
    const float zm = fmaxf((float)(iz - sd.rec_z0) * a.h, 0.5f * a.h);
    __syncthreads();
    for (int j = threadIdx.x; j < kEpiTile + 2 * HM; j += kEpiTile) {
      const int xx = x0 - HM + j;
      float e = 0.0f, A = 0.0f;
      if (xx >= 0 && xx < d.nx) {
        e = Es[xx] * a.inv_dt3;
        if (a.rcv_none) {
          A = 1.0f;
        } else {
          const float xm = (float)xx * a.h;
          A = asinhf((sd.xmax_m - xm) / zm) - asinhf((sd.xmin_m - xm) / zm);
        }
      }
      shE[j] = e;
      shA[j] = A;
    }
    __syncthreads();
    // slice h: E at x+h (LDS index tid + HM + h), A at x-h (tid + HM - h)
#pragma unroll
    for (int h = -HM; h <= HM; ++h)
      if (h >= -H && h <= H)
        acc[h + HM] = fmaf(shE[threadIdx.x + HM + h], shA[threadIdx.x + HM - h], acc[h + HM]);
  }
  if (!in || bad) return;
  if (a.H1) a.H1[cell] += h1;
  if (a.D) {
    const float vv = a.v[cell];
    const float v2 = vv * vv;
    const float fac = 4.0f / (v2 * v2 * v2);
#pragma unroll
    for (int h = -HM; h <= HM; ++h)
      if (h >= -H && h <= H) a.D[(int64_t)(h + H) * d.model + cell] += fac * acc[h + HM];
  }
}

__global__ void k_gradient_out(Dims d, const float* gacc, int S, const float* v, const double* scale,
                               double fac, float* grad, const int32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.model) return;
  float s = 0.0f;
  for (int k = 0; k < S; ++k) s += gacc[(int64_t)k * d.model + i];
  const double vv = v[i];
  const double sc = (scale ? *scale : 1.0) * fac;
  grad[i] = (*err) ? NAN : (float)(sc * 2.0 / (vv * vv * vv) * (double)s);
}

__global__ void k_traces_out(const float* traces, int ntrace, int nt_max, const ShotDesc* shots,
                             const int32_t* trace_shot, float* data) {
  const int tr = blockIdx.x;
  const int nt = shots[trace_shot[tr]].nt;
  for (int t = threadIdx.x; t < nt_max; t += blockDim.x)
    data[(int64_t)tr * nt_max + t] = (t >= 1 && t < nt) ? traces[(int64_t)t * ntrace + tr] : 0.0f;
}

__global__ void k_precond_p(int64_t n, const float* v, int kind, const float* hdiag, int nh,
                            float* out, uint32_t* maxbits) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float p = 0.0f;
  if (i < n) {
    if (kind == 0) {
      const double vv = v[i];
      p = (float)(4.0 / (vv * vv * vv * vv * vv * vv) * (double)hdiag[i]);
    } else {
      for (int h = 0; h < nh; ++h) p += hdiag[(int64_t)h * n + i];
    }
    out[i] = p;
  }
  // non-negative floats order like their bit patterns
  __shared__ uint32_t m;
  if (threadIdx.x == 0) m = 0u;
  __syncthreads();
  atomicMax(&m, __float_as_uint(fmaxf(p, 0.0f)));
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(maxbits, m);
}

__global__ void k_precond_apply(int64_t n, const float* grad, float eps, const uint32_t* maxbits,
                                float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float wl = eps * __uint_as_float(*maxbits);
  out[i] = grad[i] / (out[i] + wl);
}

// -------------------------------------------------------------------------
// launchers
// -------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

static inline unsigned step_blocks(const Dims& d, int S) {
  const int T = d.XT * d.ZT;
  const int bps = (T + kWavesPerBlock - 1) / kWavesPerBlock;
  return (unsigned)(bps * S);
}

hipError_t launch_prep(const Dims& d, const float* v, float* w, double dt, double h, float vmax,
                       int32_t* err, hipStream_t s) {
  const double dt2_h2 = dt * dt / (h * h);
  hipLaunchKernelGGL(k_prep, dim3(blocks_for(d.field, 256)), dim3(256), 0, s, d, v, w, dt2_h2, vmax,
                     err);
  return hipGetLastError();
}

hipError_t launch_prep_born(const Dims& d, const float* v, const float* dv, float* bw, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_born, dim3(blocks_for(d.field, 256)), dim3(256), 0, s, d, v, dv, bw);
  return hipGetLastError();
}

hipError_t launch_fill(void* p, size_t nbytes, hipStream_t s) {
  const size_t n = nbytes / 4;
  if (n == 0) return hipSuccess;
  const unsigned b = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fill, dim3(b), dim3(256), 0, s, (uint32_t*)p, n);
  return hipGetLastError();
}

hipError_t launch_fill_slots(float* base, int64_t stride, int64_t count, const SlotInfo* slots,
                             int S, int use_cs, hipStream_t s) {
  if (S <= 0 || count <= 0) return hipSuccess;
  const unsigned bx = (unsigned)std::min<int64_t>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_slots, dim3(bx, S), dim3(256), 0, s, base, stride, count, slots, use_cs);
  return hipGetLastError();
}

// the free-surface variant is a separate instantiation, so that the sweeps
// without one carry no trace of it
template <int FLAGS, int PF>
static void forward_fs(const StepArgs& a, hipStream_t s) {
  const dim3 grid(step_blocks(a.d, a.S)), block(256);
  if (a.d.fs) hipLaunchKernelGGL((k_forward<FLAGS | kFwdFS, PF>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_forward<FLAGS, PF>), grid, block, 0, s, a);
}

template <int PF>
static hipError_t launch_forward_pf(const StepArgs& a, int flags, hipStream_t s) {
  switch (flags) {
    case kFwdRecord: forward_fs<kFwdRecord, PF>(a, s); break;
    case kFwdRecord | kFwdCkpt: forward_fs<kFwdRecord | kFwdCkpt, PF>(a, s); break;
    case kFwdIllum: forward_fs<kFwdIllum, PF>(a, s); break;
    case kFwdRecord | kFwdBorn: forward_fs<kFwdRecord | kFwdBorn, PF>(a, s); break;
    case kFwdRecord | kFwdCkpt | kFwdBorn: forward_fs<kFwdRecord | kFwdCkpt | kFwdBorn, PF>(a, s); break;
    case kFwdCapD: forward_fs<kFwdCapD, PF>(a, s); break;
    case kFwdCapU: forward_fs<kFwdCapU, PF>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_forward(const StepArgs& a, int flags, int prefetch, hipStream_t s) {
  if ((flags & kFwdBorn) && (!a.bu || !a.bw)) return hipErrorInvalidValue;
  if ((flags & (kFwdCapD | kFwdCapU)) && !a.cap) return hipErrorInvalidValue;
  switch (prefetch) {
    case 1: return launch_forward_pf<1>(a, flags, s);
    case 3: return launch_forward_pf<3>(a, flags, s);
    case 7: return launch_forward_pf<7>(a, flags, s);
    default: return hipErrorInvalidValue;
  }
}

template <int PF, bool EXT, bool IMGU>
static void reverse_fs(const StepArgs& a, hipStream_t s) {
  const dim3 grid(step_blocks(a.d, a.S)), block(256);
  if (a.d.fs) hipLaunchKernelGGL((k_reverse<PF, EXT, IMGU, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_reverse<PF, EXT, IMGU, false>), grid, block, 0, s, a);
}

hipError_t launch_reverse(const StepArgs& a, int prefetch, int flags, hipStream_t s) {
  if ((flags & kRevExt) && (!a.ext_lam || !a.ext_D || a.ext_T < 1)) return hipErrorInvalidValue;
  if (flags < 0 || flags > 2) return hipErrorInvalidValue;
  switch (prefetch * 4 + flags) {
    case 4: reverse_fs<1, false, false>(a, s); break;
    case 5: reverse_fs<1, true, false>(a, s); break;
    case 6: reverse_fs<1, false, true>(a, s); break;
    case 12: reverse_fs<3, false, false>(a, s); break;
    case 13: reverse_fs<3, true, false>(a, s); break;
    case 14: reverse_fs<3, false, true>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_forward2(const StepArgs& a, int prefetch, hipStream_t s) {
  const dim3 grid(step_blocks(a.d, a.S)), block(256);
  if (prefetch == 3) hipLaunchKernelGGL(k_forward2<3>, grid, block, 0, s, a);
  else hipLaunchKernelGGL(k_forward2<1>, grid, block, 0, s, a);
  return hipGetLastError();
}

// one block row per slot: a shot of nt samples ran nt/2 two-step launches
// (rounded down: ceil((nt-1)/2)); with an odd count its state is in set 1
__global__ void k_forward2_finish(float* u, int64_t ustride, int64_t set_floats, const SlotInfo* slots,
                                  const ShotDesc* shots) {
  const SlotInfo si = slots[blockIdx.y];
  if (si.shot < 0) return;
  if (((shots[si.shot].nt / 2) & 1) == 0) return;
  float* base = u + (int64_t)si.cs * ustride;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < set_floats;
       k += (int64_t)gridDim.x * blockDim.x)
    base[k] = base[set_floats + k];
}

hipError_t launch_forward2_finish(float* u, int64_t ustride, int64_t set_floats, const SlotInfo* slots,
                                  const ShotDesc* shots, int S, hipStream_t s) {
  if (S <= 0 || set_floats <= 0) return hipSuccess;
  const unsigned bx = (unsigned)std::min<int64_t>((set_floats + 255) / 256, 1024);
  hipLaunchKernelGGL(k_forward2_finish, dim3(bx, S), dim3(256), 0, s, u, ustride, set_floats, slots, shots);
  return hipGetLastError();
}

hipError_t launch_reverse2(const StepArgs& a, int prefetch, int flags, hipStream_t s) {
  const dim3 grid(step_blocks(a.d, a.S)), block(256);
  const bool ext = (flags & kRevExt) != 0;
  if (prefetch == 3) {
    if (ext) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reverse2<3, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reverse2<3, false>), grid, block, 0, s, a);
  } else {
    if (ext) hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reverse2<1, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reverse2<1, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_ext_image(const ExtArgs& a, hipStream_t s) {
  const int XTm = (a.d.nx + kWave - 1) / kWave;
  const dim3 grid(blocks_for((int64_t)a.d.nz * XTm, kWavesPerBlock)), block(256);
  if (a.hmax < 0 || a.T < 1 || a.count < 1 || a.groups < 1) return hipErrorInvalidValue;
  if (a.hmax <= 16) {
    const int XTw = (a.d.nx + 4 * kWave - 1) / (4 * kWave);
    const dim3 g4(blocks_for((int64_t)a.d.nz * XTw * a.groups, kWavesPerBlock));
    if (a.hmax <= 4) hipLaunchKernelGGL(k_ext_image4<4>, g4, block, 0, s, a);
    else if (a.hmax <= 8) hipLaunchKernelGGL(k_ext_image4<8>, g4, block, 0, s, a);
    else hipLaunchKernelGGL(k_ext_image4<16>, g4, block, 0, s, a);
  } else if (a.hmax <= 32) {
    if (a.groups != 1) return hipErrorInvalidValue;  // one wavefront per column tile takes every slot
    hipLaunchKernelGGL(k_ext_image<32>, grid, block, 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ext_out(const Dims& d, const float* Iacc, int groups, int hmax, const float* v, float* image,
                          const int32_t* err, hipStream_t s) {
  const int nh = 2 * hmax + 1;
  hipLaunchKernelGGL(k_ext_out, dim3(blocks_for(d.model * nh, 256)), dim3(256), 0, s, d, Iacc, groups, nh, v,
                     image, err);
  return hipGetLastError();
}

hipError_t launch_advance(int32_t* ctr, int32_t by, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, ctr, by);
  return hipGetLastError();
}

hipError_t launch_set(int32_t* ctr, int32_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, s, ctr, value);
  return hipGetLastError();
}

hipError_t launch_misfit(const MisfitArgs& a, int S, int max_nrec, hipStream_t s) {
  if (S <= 0 || max_nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_misfit, dim3(blocks_for(max_nrec, 64), S), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce_J(const double* part, int n, double* J, const int32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_J, dim3(1), dim3(1024), 0, s, part, n, J, err);
  return hipGetLastError();
}

hipError_t launch_epilogue(const EpiArgs& a, hipStream_t s) {
  const dim3 grid(blocks_for(a.d.nx, kEpiTile), a.d.nz), block(kEpiTile);
  if (a.hmax <= 4) hipLaunchKernelGGL(k_epilogue<4>, grid, block, 0, s, a);
  else if (a.hmax <= 16) hipLaunchKernelGGL(k_epilogue<16>, grid, block, 0, s, a);
  else if (a.hmax <= 64) hipLaunchKernelGGL(k_epilogue<64>, grid, block, 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gradient_out(const Dims& d, const float* gacc, int S, const float* v,
                               const double* scale, double fac, float* grad, const int32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_gradient_out, dim3(blocks_for(d.model, 256)), dim3(256), 0, s, d, gacc, S, v,
                     scale, fac, grad, err);
  return hipGetLastError();
}

hipError_t launch_traces_out(const float* traces, int ntrace, int nt_max, const ShotDesc* shots,
                             const int32_t* trace_shot, float* data, hipStream_t s) {
  if (ntrace <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_traces_out, dim3(ntrace), dim3(256), 0, s, traces, ntrace, nt_max, shots,
                     trace_shot, data);
  return hipGetLastError();
}

hipError_t launch_precond(int nz, int nx, const float* v, const float* grad, int kind,
                          const float* hdiag, int hmax, float eps, float* out, uint32_t* maxbits,
                          hipStream_t s) {
  const int64_t n = (int64_t)nz * nx;
  hipError_t e = launch_fill(maxbits, 4, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_precond_p, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, v, kind, hdiag,
                     2 * hmax + 1, out, maxbits);
  hipLaunchKernelGGL(k_precond_apply, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, grad, eps,
                     maxbits, out);
  return hipGetLastError();
}


// -------------------------------------------------------------------------
// Offset diagonal with the exact receiver term: the offset sums of the
// summed power spectra of the two sides (the spectra themselves come from
// the matrix-core kernels of fwi_dft.hip).
// -------------------------------------------------------------------------
// one thread per model cell, the 2 HM + 1 offset sums in registers (offsets
// above hmax are skipped); PA is read at x + h, PB at x - h along the row
template <int HM>
__global__ void k_diag_products(const float* PA, const float* PB, int64_t ldp, int K, int nyq, int nz, int nx,
                                int hmax, const float* v, float scale, float* D, const int32_t* err) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, z = blockIdx.y;
  if (x >= nx || *err) return;
  const int64_t model = (int64_t)nz * nx;
  const int64_t row = (int64_t)z * nx;
  float acc[2 * HM + 1];
#pragma unroll
  for (int j = 0; j < 2 * HM + 1; ++j) acc[j] = 0.0f;
  for (int k = 0; k < K; ++k) {
    const float mk = (k == 0 || (nyq && k == K - 1)) ? 1.0f : 2.0f;
    const float* pa = PA + k * ldp + row;
    const float* pb = PB + k * ldp + row;
#pragma unroll
    for (int j = 0; j < 2 * HM + 1; ++j) {
      const int h = j - HM;
      if (h < -hmax || h > hmax || x + h < 0 || x + h >= nx || x - h < 0 || x - h >= nx) continue;
      acc[j] = fmaf(mk * pa[x + h], pb[x - h], acc[j]);
    }
  }
  const float iv = 1.0f / v[row + x];
  const float iv2 = iv * iv;
  const float f = scale * iv2 * iv2 * iv2;
#pragma unroll
  for (int j = 0; j < 2 * HM + 1; ++j) {
    const int h = j - HM;
    if (h < -hmax || h > hmax) continue;
    float* out = D + (int64_t)(h + hmax) * model + row + x;
    *out += f * acc[j];
  }
}

hipError_t launch_diag_products(const float* PA, const float* PB, int64_t ldp, int K, int nyq, int nz, int nx,
                                int hmax, const float* v, float scale, float* D, const int32_t* err,
                                hipStream_t s) {
  if (nz <= 0 || nx <= 0) return hipSuccess;
  if (ldp < (int64_t)nz * nx) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((nx + 127) / 128), (unsigned)nz), block(128);
  if (hmax <= 4)
    hipLaunchKernelGGL(k_diag_products<4>, grid, block, 0, s, PA, PB, ldp, K, nyq, nz, nx, hmax, v, scale, D,
                       err);
  else if (hmax <= 8)
    hipLaunchKernelGGL(k_diag_products<8>, grid, block, 0, s, PA, PB, ldp, K, nyq, nz, nx, hmax, v, scale, D,
                       err);
  else if (hmax <= 16)
    hipLaunchKernelGGL(k_diag_products<16>, grid, block, 0, s, PA, PB, ldp, K, nyq, nz, nx, hmax, v, scale, D,
                       err);
  else if (hmax <= 32)
    hipLaunchKernelGGL(k_diag_products<32>, grid, block, 0, s, PA, PB, ldp, K, nyq, nz, nx, hmax, v, scale, D,
                       err);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace fwi
