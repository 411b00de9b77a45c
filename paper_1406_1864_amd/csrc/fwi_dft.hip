// gfx950 matrix-core kernels of the offset-Hessian diagonal with the exact
// receiver term (section 3: the diagonal part of the subsurface-offset
// Hessian kept frequency by frequency, with the receivers' Green's
// functions).  Each forward run (a shot, or the impulse response of a
// receiver) captures the series of every model cell; the spectra of those
// series are a dense contraction with the DFT matrix,
//
//   C[c][cell] = sum_t W[c][t] X[t][cell],   W[2k][t] = cos(2 pi k t / L),
//                                            W[2k+1][t] = sin(2 pi k t / L),
//
// accumulated chunk by chunk of the record, and the summed power
// P[k][cell] += C[2k][cell]^2 + C[2k+1][cell]^2 of every run is folded into
// the last chunk's epilogue.
//
// Tiling (one workgroup of 8 wavefronts per CU, 144 KB of LDS):
//   * a workgroup owns 256 columns c (128 bins) x 256 cells and loops over
//     the runs of the launch and over the chunk's slabs of 32 time steps;
//     wavefront w computes 128 columns x 64 cells as 8 x 4 tiles of 16 x 16
//     with v_mfma_f32_16x16x32_bf16 (or v_mfma_f32_16x16x4_f32), so that each
//     column operand read from LDS feeds 4 tiles and each cell operand 8;
//   * slabs are double-buffered in LDS and the series' loads are issued one
//     slab ahead into registers: while the matrix cores work on slab j, the
//     loads of slab j+1 are in flight, one barrier per slab (two slabs in
//     flight would not fit the 256 registers the tile leaves);
//   * the DFT matrix never crosses HBM or L2 in the loop: each slab's 256
//     columns are generated into LDS from a fixed table of the 32 in-slab
//     phases (held in registers) and one phase per bin and slab;
//   * the series arrive time-major (cells contiguous, as the sweep writes
//     them); each thread gathers 16 time steps of one cell and stores them
//     cell-major into LDS, so that every MFMA operand is one 16-byte LDS read
//     per lane; rows are padded to 144 bytes (conflict-free 16-byte reads);
//   * the bf16 split keeps x = hi + lo (hi = bf16(x), lo = bf16(x - hi)) for
//     both operands and sums hi*hi + lo*hi + hi*lo with FP32 accumulation
//     (the dropped lo*lo term is about 2^-16 of the product); series and
//     DFT matrix are split on their way into LDS;
//   * the workgroups of one cell tile (its column tiles) get consecutive ids
//     on one XCD, so they stream the same series slabs from that XCD's L2.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fwi_internal.h"

namespace fwi {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;
constexpr int kPitch = 144;                       // LDS bytes per operand row (128 + 16 pad)
constexpr int kStageW = kDftCols * kPitch;        // one slab of the DFT matrix in LDS
constexpr int kStageX = kDftCells * kPitch;       // one slab of the series in LDS

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// x0, x1 split into bf16 pairs hi = bf16(x) and lo = bf16(x - hi), both
// rounded to nearest even (v_cvt_pk_bf16_f32), each packed as two halves of
// a 32-bit word (x0 in the low half)
__device__ __forceinline__ void split2(float x0, float x1, uint32_t& hi, uint32_t& lo) {
  const bf16x2 h = __builtin_convertvector((floatx2){x0, x1}, bf16x2);
  const floatx2 hv = __builtin_convertvector(h, floatx2);
  const bf16x2 l = __builtin_convertvector((floatx2){x0 - hv[0], x1 - hv[1]}, bf16x2);
  hi = __builtin_bit_cast(uint32_t, h);
  lo = __builtin_bit_cast(uint32_t, l);
}

template <bool SPLIT>
__global__ __launch_bounds__(kThreads) void k_dft(DftArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[2][kStageW + kStageX];  // [buffer][W | X]
  const int nbt = a.Cp / kDftCols;
  const int b = blockIdx.x, xcd = b & 7, q = b >> 3;
  const int bt = q % nbt, ct = (q / nbt) * 8 + xcd;
  if (ct >= a.ntile) return;  // whole workgroup: no barrier is left waiting
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wc = wave & 1, wn = wave >> 1;        // 128-column half, 64-cell quarter
  const int lr = lane & 15, lq = lane >> 4;       // MFMA row / k group of the lane
  const int64_t cell0 = (int64_t)ct * kDftCells;
  const int c0 = bt * kDftCols;

  // The DFT matrix is generated into LDS slab by slab: with t = t0 + tau
  // (t0 = 32 J the slab's first step, tau < 32),
  //   cos(a + b) = cos a cos b - sin a sin b,  sin(a + b) = sin a cos b + cos a sin b,
  // a = 2 pi k t0 / L from the per-slab phase table, b = 2 pi k tau / L from
  // the fixed table, which each thread keeps in registers for its bin k and
  // its 8 steps tau.  No twiddle crosses HBM or L2 inside the loop.
  const int wk = tid >> 2, wt = (tid & 3) * 8;   // generator role: bin (local), first tau
  const int kg = c0 / 2 + wk;                     // its global bin
  float tcos[8], tsin[8];
  {
    const float4* tb = (const float4*)(a.Tb + ((int64_t)kg * kDftKT + wt));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 v = tb[i];  // (cos, sin) of two consecutive tau
      tcos[2 * i] = v.x;
      tsin[2 * i] = v.y;
      tcos[2 * i + 1] = v.z;
      tsin[2 * i + 1] = v.w;
    }
  }
  // loader role: X - 16 of the slab's 32 steps of one cell
  const int xc = tid & (kDftCells - 1), xq = __builtin_amdgcn_readfirstlane(tid >> 8);  // xq: per wavefront
  const int64_t gcell = cell0 + xc;
  const bool cell_ok = gcell < a.model;
  struct Stage {
    float x[16];
    float2 ph;  // (cos, sin) of the slab's phase for bin kg
  };
  Stage s0;  // the next slab's loads, in flight while the current slab is multiplied

  // loads go through buffer resources with a wave-uniform base (the slab's
  // rows of this wave, the slab's phases of the workgroup's bins), a per-lane
  // offset fixed for the kernel and a uniform row offset, so that no address
  // is computed per lane in the loop
  const uint32_t xoff = (uint32_t)(cell_ok ? xc : 0) * 4u;
  const uint32_t poff = (uint32_t)wk * 8u;
  const int rows_bytes = (int)min<int64_t>(INT32_MAX, 16 * a.R * 4);  // the 16 rows a thread loads
  auto load = [&](Stage& st, int slot, int jr) {
    const int j = min(jr, a.nslab - 1);
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float2*>(a.Ph + (int64_t)(a.j0 + j) * a.Kp + c0 / 2), (short)0, kDftCols / 2 * 8, 0x00020000);
    st.ph = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rp, (int)poff, 0, 0));
    // rows t0 .. t0 + 15 of this wave, clamped to the chunk's last step
    const int t0 = min(j * kDftKT + 16 * xq, a.tc - 1);
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(a.X + (int64_t)slot * a.xslot + (int64_t)t0 * a.R + cell0), (short)0, rows_bytes,
        0x00020000);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int r = min(t0 + i, a.tc - 1) - t0;
      st.x[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, (int)xoff, (int)(r * a.R * 4), 0));
    }
  };
  auto store = [&](Stage& st, int buf, int j) {
    const int t0 = j * kDftKT + 16 * xq;
#pragma unroll
    for (int i = 0; i < 16; ++i) st.x[i] = (cell_ok && t0 + i < a.tc) ? st.x[i] : 0.0f;
    uint8_t* A = lds[buf];
    uint8_t* B = lds[buf] + kStageW;
    // rows 2 wk (cosine) and 2 wk + 1 (sine), steps wt .. wt + 7
    float wc8[8], ws8[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      wc8[i] = fmaf(st.ph.x, tcos[i], -st.ph.y * tsin[i]);
      ws8[i] = fmaf(st.ph.y, tcos[i], st.ph.x * tsin[i]);
    }
    uint8_t* rc = A + (2 * wk) * kPitch;
    uint8_t* rs = rc + kPitch;
    uint8_t* row = B + xc * kPitch;
    if (SPLIT) {
      uint32_t ch[4], cl[4], sh[4], sl[4], xh[8], xl[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        split2(wc8[2 * i], wc8[2 * i + 1], ch[i], cl[i]);
        split2(ws8[2 * i], ws8[2 * i + 1], sh[i], sl[i]);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) split2(st.x[2 * i], st.x[2 * i + 1], xh[i], xl[i]);
      *(uint4*)(rc + 2 * wt) = make_uint4(ch[0], ch[1], ch[2], ch[3]);
      *(uint4*)(rc + 64 + 2 * wt) = make_uint4(cl[0], cl[1], cl[2], cl[3]);
      *(uint4*)(rs + 2 * wt) = make_uint4(sh[0], sh[1], sh[2], sh[3]);
      *(uint4*)(rs + 64 + 2 * wt) = make_uint4(sl[0], sl[1], sl[2], sl[3]);
      *(uint4*)(row + 32 * xq) = make_uint4(xh[0], xh[1], xh[2], xh[3]);
      *(uint4*)(row + 32 * xq + 16) = make_uint4(xh[4], xh[5], xh[6], xh[7]);
      *(uint4*)(row + 64 + 32 * xq) = make_uint4(xl[0], xl[1], xl[2], xl[3]);
      *(uint4*)(row + 64 + 32 * xq + 16) = make_uint4(xl[4], xl[5], xl[6], xl[7]);
    } else {
      *(float4*)(rc + 4 * wt) = make_float4(wc8[0], wc8[1], wc8[2], wc8[3]);
      *(float4*)(rc + 4 * wt + 16) = make_float4(wc8[4], wc8[5], wc8[6], wc8[7]);
      *(float4*)(rs + 4 * wt) = make_float4(ws8[0], ws8[1], ws8[2], ws8[3]);
      *(float4*)(rs + 4 * wt + 16) = make_float4(ws8[4], ws8[5], ws8[6], ws8[7]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        *(float4*)(row + 64 * xq + 16 * i) = make_float4(st.x[4 * i], st.x[4 * i + 1], st.x[4 * i + 2], st.x[4 * i + 3]);
    }
  };

  floatx4 acc[8][4];
  auto compute = [&](int buf) {
    const uint8_t* A = lds[buf] + (wc * 128 + lr) * kPitch;
    const uint8_t* B = lds[buf] + kStageW + (wn * 64 + lr) * kPitch;
    if (SPLIT) {
      bf16x8 bh[4], bl[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        bh[n] = __builtin_bit_cast(bf16x8, *(const uint4*)(B + n * 16 * kPitch + lq * 16));
        bl[n] = __builtin_bit_cast(bf16x8, *(const uint4*)(B + n * 16 * kPitch + 64 + lq * 16));
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, *(const uint4*)(A + m * 16 * kPitch + lq * 16));
        const bf16x8 al = __builtin_bit_cast(bf16x8, *(const uint4*)(A + m * 16 * kPitch + 64 + lq * 16));
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[n], acc[m][n], 0, 0, 0);
          acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[n], acc[m][n], 0, 0, 0);
          acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[n], acc[m][n], 0, 0, 0);
        }
      }
    } else {
      // k group lq of MFMA s takes step 8 lq + s of the slab: every lane's
      // eight operands of one tile are contiguous
      float4 bv[4][2];
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        bv[n][0] = *(const float4*)(B + n * 16 * kPitch + lq * 32);
        bv[n][1] = *(const float4*)(B + n * 16 * kPitch + lq * 32 + 16);
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const float4 a0 = *(const float4*)(A + m * 16 * kPitch + lq * 32);
        const float4 a1 = *(const float4*)(A + m * 16 * kPitch + lq * 32 + 16);
        const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          const float bw[8] = {bv[n][0].x, bv[n][0].y, bv[n][0].z, bv[n][0].w,
                               bv[n][1].x, bv[n][1].y, bv[n][1].z, bv[n][1].w};
#pragma unroll
          for (int s = 0; s < 8; ++s) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bw[s], acc[m][n], 0, 0, 0);
        }
      }
    }
  };

  for (int slot = 0; slot < a.nslots; ++slot) {
    // the first two slabs' loads go out before the running spectra's
    load(s0, slot, 0);
    // the run's spectra, lane row pointer: the wavefront's 16 rows (m, i)
    // are walked by pointer increments, its 4 cell tiles are immediate offsets
    float* Cs = a.C + (int64_t)slot * a.Cp * a.R + (int64_t)(c0 + wc * 128 + 4 * lq) * a.R + cell0 + wn * 64 + lr;
    if (a.first) {
#pragma unroll
      for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    } else {
      const float* row = Cs;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
          for (int n = 0; n < 4; ++n) acc[m][n][i] = row[n * 16];
          row += a.R;
        }
        row += 12 * a.R;
      }
    }
    store(s0, 0, 0);
    __syncthreads();
    // slab j is in LDS buffer j & 1; slab j + 1 is loaded into registers
    // while slab j is multiplied, and stored into the other buffer after it
    for (int j = 0; j < a.nslab; ++j) {
      const bool more = j + 1 < a.nslab;
      if (more) load(s0, slot, j + 1);
      compute(j & 1);
      if (more) store(s0, (j + 1) & 1, j + 1);
      __syncthreads();
    }
    // epilogue: the spectra, or after the run's last chunk their powers
    if (!a.last) {
      float* row = Cs;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
          for (int n = 0; n < 4; ++n) row[n * 16] = acc[m][n][i];
          row += a.R;
        }
        row += 12 * a.R;
      }
    } else {
      // rows 2p, 2p + 1 of the lane's four are the cosine and sine of bin
      // kb + 8 m + p (P is padded to Kp bins x R cells: no lane is masked);
      // all 32 running sums of the lane are read before any is written back
      const int kb = (c0 + wc * 128 + 4 * lq) / 2;
      float* const p0 = a.P + (int64_t)kb * a.R + cell0 + wn * 64 + lr;
      float old[8][2][4];
#pragma unroll
      for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int n = 0; n < 4; ++n) old[m][p][n] = p0[(int64_t)(8 * m + p) * a.R + n * 16];
#pragma unroll
      for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int n = 0; n < 4; ++n) {
            const floatx4& c = acc[m][n];
            p0[(int64_t)(8 * m + p) * a.R + n * 16] =
                fmaf(c[2 * p], c[2 * p], fmaf(c[2 * p + 1], c[2 * p + 1], old[m][p][n]));
          }
    }
  }
}

// (cos, sin)(2 pi r / L) of the phase r = k t mod L, reduced exactly in
// integers, the angle in double
__device__ __forceinline__ float2 phase(int64_t k, int64_t t, int L) {
  const int64_t r = (k * t) % L;
  double sn, cs;
  sincospi(2.0 * (double)r / (double)L, &sn, &cs);
  return make_float2((float)cs, (float)sn);
}

// Tb[k][tau] = phase(k, tau), tau < 32; Ph[J][k] = phase(k, 32 J), J < nslab;
// zero for bins k >= K (the DFT matrix's padding columns)
__global__ void k_dft_tables(float2* Tb, float2* Ph, int nslab, int Kp, int K, int L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)Kp * kDftKT;
  if (i < nt) {
    const int k = (int)(i / kDftKT), tau = (int)(i % kDftKT);
    Tb[i] = k < K ? phase(k, tau, L) : make_float2(0.0f, 0.0f);
  } else if (i < nt + (int64_t)nslab * Kp) {
    const int64_t e = i - nt;
    const int J = (int)(e / Kp), k = (int)(e % Kp);
    Ph[e] = k < K ? phase(k, (int64_t)J * kDftKT, L) : make_float2(0.0f, 0.0f);
  }
}

}  // namespace

hipError_t launch_dft(const DftArgs& a, int split, hipStream_t s) {
  if (a.nslots <= 0 || a.ntile <= 0 || a.nslab <= 0) return hipSuccess;
  if (a.Cp <= 0 || a.Cp % kDftCols || 2 * a.Kp != a.Cp || a.R != (int64_t)a.ntile * kDftCells || a.R < a.model ||
      a.tc > a.nslab * kDftKT || a.tc <= (a.nslab - 1) * kDftKT || 2 * a.K > a.Cp)
    return hipErrorInvalidValue;
  const int64_t blocks = (int64_t)((a.ntile + 7) / 8) * 8 * (a.Cp / kDftCols);
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  if (split)
    hipLaunchKernelGGL(k_dft<true>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_dft<false>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_dft_tables(float2* Tb, float2* Ph, int nslab, int Kp, int K, int L, hipStream_t s) {
  if (nslab <= 0 || Kp <= 0) return hipSuccess;
  if (K > Kp || L <= 0) return hipErrorInvalidValue;
  const int64_t n = (int64_t)Kp * kDftKT + (int64_t)nslab * Kp;
  hipLaunchKernelGGL(k_dft_tables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Tb, Ph, nslab, Kp, K, L);
  return hipGetLastError();
}

}  // namespace fwi
