// Ablation: the raw-moment transform as a dense matrix product on MFMA (D3Q27, pull).
//
// The Chimera passes of the default sweep evaluate m = M df with 81 additions per cell
// (eq. RawMomentChimeraTransform, sec. 4.1.1).  Here the same m = M df and df* = M^-1 dm*
// are computed as dense 27 x 27 products over the 64 cells of a wave with
// v_mfma_{f32,f64}_16x16x4: rows padded to 32 (two 16-row tiles), the contraction padded to
// 28 (seven K-steps of 4), the 64 cells as four 16-column tiles.  Columns are exchanged
// through LDS (a [27][65] region per wave: cell-major in, MFMA fragments out).  Everything
// between the two transforms is the same collide_moments as the default kernel, so the
// kernel measures the cost of replacing the Chimera with MFMA and LDS traffic.
//
// MFMA 16x16x4 operand layout (one value per lane for A and B, four for D), checked on gfx950:
//   A[i][k] in lane i + 16 k,  B[k][j] in lane j + 16 k;
//   f32: D[i][j] in lane j + 16 (i / 4), register i % 4;
//   f64: D[i][j] in lane j + 16 (i % 4), register i / 4.
#pragma once

#include "lbm_kernels.hpp"

namespace lbm {

template <class CT> struct Mfma;
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of D held by register r of a lane in row group lk = lane / 16
  static __device__ __forceinline__ int drow(int lk, int r) { return 4 * lk + r; }
};
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lk, int r) { return 4 * r + lk; }
};

constexpr int MFMA_LDS_STRIDE = 65;  // padded row of 64 cells (avoids bank conflicts)
constexpr int MFMA_ROWS = 27;

// entries of M (moment e from velocity k) and M^-1 (velocity k from moment e); both index
// spaces are the 3x3x3 grids: e = a + 3b + 9c (exponents), k = (cx+1) + 3(cy+1) + 9(cz+1)
template <class CT>
__device__ __forceinline__ CT mono_entry(int e, int k) {
  if (e >= 27 || k >= 27) return CT(0);
  CT v = CT(1);
  int ee = e, kk = k;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ex = ee % 3, c = kk % 3 - 1;
    ee /= 3;
    kk /= 3;
    v *= ex == 0 ? CT(1) : (ex == 1 ? CT(c) : CT(c * c));
  }
  return v;
}
template <class CT>
__device__ __forceinline__ CT inv_entry(int k, int e) {
  if (e >= 27 || k >= 27) return CT(0);
  // 1-D inverse: f_-1 = (m2 - m1)/2, f_0 = m0 - m2, f_+1 = (m2 + m1)/2
  CT v = CT(1);
  int ee = e, kk = k;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ex = ee % 3, c = kk % 3 - 1;
    ee /= 3;
    kk /= 3;
    CT w;
    if (c == 0) w = ex == 0 ? CT(1) : (ex == 1 ? CT(0) : CT(-1));
    else w = ex == 0 ? CT(0) : (ex == 1 ? CT(0.5) * CT(c) : CT(0.5));
    v *= w;
  }
  return v;
}

// y = A x over the 64 lanes of a wave, x and y per lane (column = lane).  INV selects M^-1.
template <bool INV, class CT>
__device__ __forceinline__ void wave_dense27(CT *x, CT *lds, int lane) {
  using V4 = typename Mfma<CT>::v4;
#pragma unroll
  for (int k = 0; k < MFMA_ROWS; ++k) lds[k * MFMA_LDS_STRIDE + lane] = x[k];
  __syncthreads();
  V4 acc[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = V4{CT(0), CT(0), CT(0), CT(0)};
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < 7; ++ks) {
    const int k = 4 * ks + lk;
    const CT a0 = INV ? inv_entry<CT>(li, k) : mono_entry<CT>(li, k);
    const CT a1 = INV ? inv_entry<CT>(16 + li, k) : mono_entry<CT>(16 + li, k);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const CT b = k < MFMA_ROWS ? lds[k * MFMA_LDS_STRIDE + 16 * ct + li] : CT(0);
      acc[0][ct] = Mfma<CT>::mma(a0, b, acc[0][ct]);
      acc[1][ct] = Mfma<CT>::mma(a1, b, acc[1][ct]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * rt + Mfma<CT>::drow(lk, r);
        if (row < MFMA_ROWS) lds[row * MFMA_LDS_STRIDE + 16 * ct + li] = acc[rt][ct][r];
      }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < MFMA_ROWS; ++k) x[k] = lds[k * MFMA_LDS_STRIDE + lane];
  __syncthreads();
}

// the ablation sweep; blocks of at most 256 threads (4 waves), LDS 27 x 65 x sizeof(CT) per wave
template <int SP, bool REG, class ST, class CT>
__global__ void __launch_bounds__(256) sweep_mfma_kernel(SweepArgs<ST, CT> a) {
  using L = Lat<D3Q27>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int lane = tid & 63;
  CT *lds = reinterpret_cast<CT *>(lds_raw) + (tid >> 6) * (MFMA_ROWS * MFMA_LDS_STRIDE);
  CellPos p = tile_cell_args(a, 1);
  // lanes outside the box still take part in the wave-wide products (with zero input)
  const bool valid = p.valid;
  if (!valid) {
    p.x = 0;
    p.y = 0;
  }
  const Nbr<3> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz, a.L);
  CT g[27];
  sfor<27>([&](auto E) { g[E] = CT(0); });
  if (valid) {
    sfor<27>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
      g[L::gidx(i)] = CT(ldp(a.src, (uint64_t(i) * a.L.ps) + nb.zpart(cz, -1), nb.lane(cx, cy, -1)));
    });
  }
  if (a.absolute && valid) sfor<27>([&](auto I) { g[L::gidx(I)] -= CT(L::w(I)); });
  wave_dense27<false, CT>(g, lds, lane);
  collide_moments<D3Q27, SP, MAXWELL, REG, CT>(g, a.R, CT(0));
  wave_dense27<true, CT>(g, lds, lane);
  if (a.absolute) sfor<27>([&](auto I) { g[L::gidx(I)] += CT(L::w(I)); });
  if (valid) {
    sfor<27>([&](auto I) {
      constexpr int i = decltype(I)::value;
      stp(a.dst, (uint64_t(i) * a.L.ps) + nb.zpart(0, 1), nb.lane(0, 0, 1), ST(g[L::gidx(i)]));
    });
  }
}

}  // namespace lbm
