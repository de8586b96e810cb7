// HIP kernels of the lattice Boltzmann library (gfx950).
//
// sweep_kernel   fused stream + collide over every cell (eq. LbUpdateScheme, sec. 2.1, with
//                the collision of sec. 2.2) for the pull and AA patterns (sec. 4.4)
// init_kernel    zero-centred equilibrium initialisation in FP64 (sec. 2.4)
// export_kernel / import_kernel   canonical df(t) <-> storage layout
// macro_kernel   density and velocity of df(t) (eq. DensityAndVelocityFromDeviation)
// diag_kernel    FP64 mass / momentum / kinetic-energy / non-finite reductions
//
// Storage is SoA: population i of cell c at buf[i * ncells + c], x fastest.  One thread owns
// one cell; a block covers bx cells along x and by rows along y of one z-plane.  Periodic
// neighbours come from per-axis wrapped coordinates (integer selects only).
#pragma once

#include "lbm_device.hpp"

namespace lbm {

enum StorageId { F64 = 0, F32 = 1, F16 = 2 };

template <int ST> struct StoreTraits;
template <> struct StoreTraits<F64> { using S = double;   using C = double; };
template <> struct StoreTraits<F32> { using S = float;    using C = float; };
template <> struct StoreTraits<F16> { using S = _Float16; using C = float; };

template <class ST, class CT>
struct SweepArgs {
  const ST *src;
  ST *dst;
  int nx, ny, nz;
  uint32_t plane;    // population plane stride in elements (plane * sizeof(ST) < 2^32)
  int tiles_x, tiles_y;
  int swizzle;       // nonzero: consecutive tiles on one XCD
  CT grav;
  Relax<CT> R;
};

// 8 XCDs receive workgroups round-robin; give each XCD a contiguous range of tiles.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
  const uint32_t per = n / 8u, rem = n % 8u;
  const uint32_t xcd = b % 8u, local = b / 8u;
  return xcd < rem ? xcd * (per + 1u) + local : rem * (per + 1u) + (xcd - rem) * per + local;
}

struct CellPos {
  int x, y, z;
  bool valid;
};

__device__ __forceinline__ CellPos tile_cell(int nx, int ny, int tiles_x, int tiles_y, int swz) {
  uint32_t tile = blockIdx.x;
  if (swz) tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint32_t per_plane = uint32_t(tiles_x) * uint32_t(tiles_y);
  const uint32_t tz = tile / per_plane;
  const uint32_t r = tile - tz * per_plane;
  const uint32_t ty = r / uint32_t(tiles_x);
  const uint32_t tx = r - ty * uint32_t(tiles_x);
  CellPos p;
  p.x = int(tx * blockDim.x + threadIdx.x);
  p.y = int(ty * blockDim.y + threadIdx.y);
  p.z = int(tz);
  p.valid = p.x < nx && p.y < ny;
  return p;
}

// neighbour tables of one cell: rows[dy+1][dz+1] = (zw * ny + yw) * nx, xs[dx+1] = xw
template <int D>
struct Nbr {
  uint32_t rows[3][3];
  uint32_t xs[3];
  __device__ __forceinline__ Nbr(int x, int y, int z, int nx, int ny, int nz) {
    xs[0] = uint32_t(x == 0 ? nx - 1 : x - 1);
    xs[1] = uint32_t(x);
    xs[2] = uint32_t(x == nx - 1 ? 0 : x + 1);
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const int yy[3] = {ym, y, yp};
    if constexpr (D == 3) {
      const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
      const int zz[3] = {zm, z, zp};
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) rows[b][c] = (uint32_t(zz[c]) * uint32_t(ny) + uint32_t(yy[b])) * uint32_t(nx);
    } else {
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const uint32_t r = (uint32_t(z) * uint32_t(ny) + uint32_t(yy[b])) * uint32_t(nx);
        rows[b][0] = r;
        rows[b][1] = r;
        rows[b][2] = r;
      }
    }
  }
  // cell at x + s * xi (s = -1 or +1) for velocity (cx, cy, cz)
  __device__ __forceinline__ uint32_t at(int cx, int cy, int cz, int s) const {
    return rows[1 + s * cy][1 + s * cz] + xs[1 + s * cx];
  }
};

template <class ST>
__device__ __forceinline__ ST ld(const ST *base, uint32_t plane, int i, uint32_t cell) {
  return base[size_t(i) * plane + cell];
}
template <class ST>
__device__ __forceinline__ void st(ST *base, uint32_t plane, int i, uint32_t cell, ST v) {
  base[size_t(i) * plane + cell] = v;
}

// ---------------------------------------------------------------------------------------
// fused stream + collide
// ---------------------------------------------------------------------------------------
template <int S, int SP, int EQ, bool REG, class ST, class CT, int PAT>
__global__ void __launch_bounds__(512) sweep_kernel(SweepArgs<ST, CT> a) {
  using L = Lat<S>;
  const CellPos p = tile_cell(a.nx, a.ny, a.tiles_x, a.tiles_y, a.swizzle);
  if (!p.valid) return;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz);
  const uint32_t self = nb.rows[1][1] + uint32_t(p.x);

  CT g[L::G];
  sfor<L::G>([&](auto E) { g[E] = CT(0); });
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
    if constexpr (PAT == PULL) {
      g[L::gidx(i)] = CT(ld(a.src, a.plane, i, nb.at(cx, cy, cz, -1)));
    } else if constexpr (PAT == AA_EVEN) {
      g[L::gidx(i)] = CT(ld(a.src, a.plane, i, self));
    } else {
      g[L::gidx(i)] = CT(ld(a.src, a.plane, L::opp(i), nb.at(cx, cy, cz, -1)));
    }
  });

  collide<S, SP, EQ, REG, CT>(g, a.R, a.grav);

  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
    const ST v = ST(g[L::gidx(i)]);
    if constexpr (PAT == PULL) {
      st(a.dst, a.plane, i, self, v);
    } else if constexpr (PAT == AA_EVEN) {
      st(a.dst, a.plane, L::opp(i), self, v);
    } else {
      st(a.dst, a.plane, i, nb.at(cx, cy, cz, +1), v);
    }
  });
}

// ---------------------------------------------------------------------------------------
// readers / writers of the canonical state
// ---------------------------------------------------------------------------------------
struct FieldArgs {
  void *buf;          // population buffer (storage type), first cell of the box
  uint32_t plane;     // population plane stride of the buffer in elements
  uint32_t ncells;    // cells of the box (stride of the FP64 field arrays)
  int nx, ny, nz;
  int tiles_x, tiles_y;
  double grav;
  const double *rho_in;   // init
  const double *u_in;
  double *rho_out;        // macroscopic
  double *u_out;
  double *pop;            // export (out) / import (in): df[i * ncells + c], FP64
  double *partials;       // diagnostics: 6 per block
  int i0, i1;             // population range of export / import (chunking)
};

// address of the canonical df_i(x) in the buffer for layout GM
template <int S, int GM>
__device__ __forceinline__ void canon_addr(const Nbr<Lat<S>::D> &nb, uint32_t self, int i, int cx, int cy, int cz,
                                           int &slot, uint32_t &cell) {
  if constexpr (GM == G_NATURAL) {
    slot = i;
    cell = self;
  } else if constexpr (GM == G_SHIFTED) {
    slot = i;
    cell = nb.at(cx, cy, cz, -1);
  } else {
    slot = Lat<S>::opp(i);
    cell = nb.at(cx, cy, cz, -1);
  }
}

template <int S, int GM, class ST>
__device__ __forceinline__ void gather_canon(const FieldArgs &a, const CellPos &p, double *f) {
  using L = Lat<S>;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz);
  const uint32_t self = nb.rows[1][1] + uint32_t(p.x);
  const ST *buf = static_cast<const ST *>(a.buf);
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    int slot;
    uint32_t cell;
    canon_addr<S, GM>(nb, self, i, L::c(i, 0), L::c(i, 1), L::c(i, 2), slot, cell);
    f[i] = double(ld(buf, a.plane, slot, cell));
  });
}

// df(0) = f_eq(rho, u) - f0, written in layout GM (G_SHIFTED for pull, G_NATURAL for AA)
template <int S, int SP, int EQ, int GM, class ST>
__global__ void __launch_bounds__(256) init_kernel(FieldArgs a) {
  using L = Lat<S>;
  const CellPos p = tile_cell(a.nx, a.ny, a.tiles_x, a.tiles_y, 0);
  if (!p.valid) return;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz);
  const uint32_t self = nb.rows[1][1] + uint32_t(p.x);
  const double drho = a.rho_in[self] - 1.0;
  double u[3] = {a.u_in[self], a.u_in[size_t(a.ncells) + self], L::D == 3 ? a.u_in[2 * size_t(a.ncells) + self] : 0.0};
  double g[L::G];
  equilibrium_dev<S, SP, EQ, double>(g, drho, u, a.grav);
  ST *buf = static_cast<ST *>(a.buf);
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    int slot;
    uint32_t cell;
    canon_addr<S, GM>(nb, self, i, L::c(i, 0), L::c(i, 1), L::c(i, 2), slot, cell);
    st(buf, a.plane, slot, cell, ST(g[L::gidx(i)]));
  });
}

template <int S, int GM, class ST>
__global__ void __launch_bounds__(256) export_kernel(FieldArgs a) {
  using L = Lat<S>;
  const CellPos p = tile_cell(a.nx, a.ny, a.tiles_x, a.tiles_y, 0);
  if (!p.valid) return;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz);
  const uint32_t self = nb.rows[1][1] + uint32_t(p.x);
  const ST *buf = static_cast<const ST *>(a.buf);
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if (i >= a.i0 && i < a.i1) {
      int slot;
      uint32_t cell;
      canon_addr<S, GM>(nb, self, i, L::c(i, 0), L::c(i, 1), L::c(i, 2), slot, cell);
      a.pop[size_t(i - a.i0) * a.ncells + self] = double(ld(buf, a.plane, slot, cell));
    }
  });
}

template <int S, int GM, class ST>
__global__ void __launch_bounds__(256) import_kernel(FieldArgs a) {
  using L = Lat<S>;
  const CellPos p = tile_cell(a.nx, a.ny, a.tiles_x, a.tiles_y, 0);
  if (!p.valid) return;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz);
  const uint32_t self = nb.rows[1][1] + uint32_t(p.x);
  ST *buf = static_cast<ST *>(a.buf);
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if (i >= a.i0 && i < a.i1) {
      int slot;
      uint32_t cell;
      canon_addr<S, GM>(nb, self, i, L::c(i, 0), L::c(i, 1), L::c(i, 2), slot, cell);
      st(buf, a.plane, slot, cell, ST(a.pop[size_t(i - a.i0) * a.ncells + self]));
    }
  });
}

template <int S, int GM, class ST>
__global__ void __launch_bounds__(256) macro_kernel(FieldArgs a) {
  using L = Lat<S>;
  const CellPos p = tile_cell(a.nx, a.ny, a.tiles_x, a.tiles_y, 0);
  if (!p.valid) return;
  double f[L::Q];
  gather_canon<S, GM, ST>(a, p, f);
  double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    drho += f[i];
    if constexpr (L::c(i, 0) != 0) j[0] += double(L::c(i, 0)) * f[i];
    if constexpr (L::c(i, 1) != 0) j[1] += double(L::c(i, 1)) * f[i];
    if constexpr (L::c(i, 2) != 0) j[2] += double(L::c(i, 2)) * f[i];
  });
  const double rho = 1.0 + drho;
  const uint32_t self = (uint32_t(p.z) * uint32_t(a.ny) + uint32_t(p.y)) * uint32_t(a.nx) + uint32_t(p.x);
  a.rho_out[self] = rho;
  a.u_out[self] = j[0] / rho;
  a.u_out[size_t(a.ncells) + self] = j[1] / rho;
  a.u_out[2 * size_t(a.ncells) + self] = j[2] / rho;
}

// grid-stride over cells in a fixed order per thread, block tree in LDS -> deterministic
constexpr int DIAG_THREADS = 256;
template <int S, int GM, class ST>
__global__ void __launch_bounds__(DIAG_THREADS) diag_kernel(FieldArgs a) {
  using L = Lat<S>;
  __shared__ double red[6][DIAG_THREADS];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const uint32_t nrow = uint32_t(a.ny) * uint32_t(a.nz);
  const uint64_t total = uint64_t(a.ncells);
  for (uint64_t c = uint64_t(blockIdx.x) * DIAG_THREADS + threadIdx.x; c < total;
       c += uint64_t(gridDim.x) * DIAG_THREADS) {
    CellPos p;
    p.x = int(c % uint64_t(a.nx));
    const uint32_t row = uint32_t(c / uint64_t(a.nx));
    p.y = int(row % uint32_t(a.ny));
    p.z = int(row / uint32_t(a.ny));
    p.valid = true;
    (void)nrow;
    double f[L::Q];
    gather_canon<S, GM, ST>(a, p, f);
    double drho = 0.0, j[3] = {0.0, 0.0, 0.0}, bad = 0.0;
    sfor<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      drho += f[i];
      bad += (__builtin_isfinite(f[i]) ? 0.0 : 1.0);
      if constexpr (L::c(i, 0) != 0) j[0] += double(L::c(i, 0)) * f[i];
      if constexpr (L::c(i, 1) != 0) j[1] += double(L::c(i, 1)) * f[i];
      if constexpr (L::c(i, 2) != 0) j[2] += double(L::c(i, 2)) * f[i];
    });
    acc[0] += drho;
    acc[1] += j[0];
    acc[2] += j[1];
    acc[3] += j[2];
    acc[4] += 0.5 * (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / (1.0 + drho);
    acc[5] += bad;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = DIAG_THREADS / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) {
#pragma unroll
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) a.partials[size_t(blockIdx.x) * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// final fixed-order sum of nblocks x 6 partials by one block
__global__ void __launch_bounds__(DIAG_THREADS) diag_final_kernel(const double *partials, int nblocks, double *out);

}  // namespace lbm
