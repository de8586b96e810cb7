// HIP kernels of the lattice Boltzmann library (gfx950).
//
// sweep_kernel   fused stream + collide over every cell (eq. LbUpdateScheme, sec. 2.1, with
//                the collision of sec. 2.2) for the pull, push, AA, Esoteric-Pull and
//                Esoteric-Twist patterns (sec. 4.4)
// init_kernel    zero-centred equilibrium initialisation in FP64 (sec. 2.4)
// export_kernel / import_kernel   canonical df(t) <-> storage layout
// macro_kernel   density and velocity of df(t) (eq. DensityAndVelocityFromDeviation)
// diag_kernel    FP64 mass / momentum / kinetic-energy / non-finite reductions
//
// Storage is SoA with x fastest, either one plane per population or the q populations of a
// row side by side (Strides).  One thread owns one cell; a block covers bx cells along x and
// by rows along y of one z-plane.  Periodic neighbours come from per-axis wrapped
// coordinates (integer selects only).  Stores are non-temporal: every population written in
// a sweep is read again only in the next sweep, after the whole 2 Q sizeof(ST) ncells bytes
// have streamed through the caches.
//
// Push (two buffers): the state between steps is the natural layout (f_i(x) at x, slot i); a
// step reads the cell's own slots and writes f*_i to x + xi in the other buffer.
//
// In-place patterns (one buffer; each step every cell reads and writes the same locations, so
// the sweep is race-free).  Directions come in opposite pairs (i odd, opp(i) = i + 1).
//   AA:            even steps use the cell's own slots (reading slot i, writing slot opp(i));
//                  odd steps read slot opp(i) at x - xi and write slot i at x + xi.
//   Esoteric Pull: every step touches the own cell and the neighbours x + xi of the odd
//                  directions only.  Odd i and the rest population live at the own cell,
//                  even i at x - xi; on even steps population i is found in slot opp(i), on
//                  odd steps in slot i.  After the collision odd directions are written to
//                  x + xi, the others stay, the slot index flipping with the parity.
//   Esoteric Twist: every step touches the nodes x + {0, 1}^3 only.  Population i lives at
//                  x + (-xi)^+ (componentwise positive part), in slot i after an even number
//                  of steps and in slot opp(i) after an odd number; after the collision it is
//                  written to x + (xi)^+ = the home node of opp(i), in the other slot.  The
//                  two step kinds differ only in the slot naming.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

enum StorageId { F64 = 0, F32 = 1, F16 = 2 };

template <int ST> struct StoreTraits;
template <> struct StoreTraits<F64> { using S = double;   using C = double; };
template <> struct StoreTraits<F32> { using S = float;    using C = float; };
template <> struct StoreTraits<F16> { using S = _Float16; using C = float; };

// Storage layout: population i of cell (x, y, z) lives at element
//   i * ps + z * zs + y * ys + x
// planes layout: ps = plane (>= ncells, padded), zs = ny * nx, ys = nx
// rows layout:   ps = nxp (nx rounded up), ys = q * nxp, zs = ny * ys  (all q populations of
//                one row side by side, so a block touches a few contiguous rows per plane)
// Per block z is uniform, so i * ps + z * zs is a scalar 64-bit base and y * ys + x the
// 32-bit per-lane offset (bounded by zs < 2^32 elements of a z-plane).
struct Strides {
  uint64_t ps, zs;
  uint32_t ys;
};

template <class ST, class CT>
struct SweepArgs {
  const ST *src;
  ST *dst;
  int nx, ny, nz;
  Strides L;
  int tiles_x, tiles_y;
  int swizzle;       // nonzero: consecutive tiles on one XCD
  int absolute;      // nonzero: buffers hold absolute populations f = df + w
  int bx, by;        // block shape (threads along x, rows along y)
  const uint2 *tile_table;  // per block: (tx | ty << 16, tz), XCD order applied; or null
  const CT *ffield;  // forced sweep: body force per cell [3][ncells] (natural order), or null
  CT fconst[3];      // forced sweep: constant body force added to ffield
  int force_model;   // forced sweep: FORCE_GUO or FORCE_HE
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

// tile of this block from the host-built table (no divisions on the device), else computed
template <class A>
__device__ __forceinline__ CellPos tile_cell_args(const A &a, int cells_per_lane) {
  uint32_t tx, ty, tz;
  if (a.tile_table) {
    const uint2 t = a.tile_table[blockIdx.x];
    tx = t.x & 0xffffu;
    ty = t.x >> 16;
    tz = t.y;
  } else {
    uint32_t tile = blockIdx.x;
    if (a.swizzle) tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t per_plane = uint32_t(a.tiles_x) * uint32_t(a.tiles_y);
    tz = tile / per_plane;
    const uint32_t r = tile - tz * per_plane;
    ty = r / uint32_t(a.tiles_x);
    tx = r - ty * uint32_t(a.tiles_x);
  }
  CellPos p;
  p.x = int((tx * uint32_t(a.bx) + threadIdx.x) * uint32_t(cells_per_lane));
  p.y = int(ty * uint32_t(a.by) + threadIdx.y);
  p.z = int(tz);
  p.valid = p.x < a.nx && p.y < a.ny;
  return p;
}

// periodic neighbours of one cell in a strided buffer
template <int D>
struct Nbr {
  uint64_t zoff[3];  // (z + dz wrapped) * zs, block-uniform
  uint32_t yoff[3];  // (y + dy wrapped) * ys
  uint32_t xs[3];    // x + dx wrapped
  __device__ __forceinline__ Nbr(int x, int y, int z, int nx, int ny, int nz, const Strides &L) {
    xs[0] = uint32_t(x == 0 ? nx - 1 : x - 1);
    xs[1] = uint32_t(x);
    xs[2] = uint32_t(x == nx - 1 ? 0 : x + 1);
    yoff[0] = uint32_t(y == 0 ? ny - 1 : y - 1) * L.ys;
    yoff[1] = uint32_t(y) * L.ys;
    yoff[2] = uint32_t(y == ny - 1 ? 0 : y + 1) * L.ys;
    if constexpr (D == 3) {
      zoff[0] = uint64_t(z == 0 ? nz - 1 : z - 1) * L.zs;
      zoff[1] = uint64_t(z) * L.zs;
      zoff[2] = uint64_t(z == nz - 1 ? 0 : z + 1) * L.zs;
    } else {
      zoff[0] = zoff[1] = zoff[2] = uint64_t(z) * L.zs;
    }
  }
  // element offset (without the population term) of the cell at x + s * xi
  __device__ __forceinline__ uint64_t zpart(int cz, int s) const { return zoff[1 + s * cz]; }
  __device__ __forceinline__ uint32_t lane(int cx, int cy, int s) const { return yoff[1 + s * cy] + xs[1 + s * cx]; }
};

// The lane part is turned into a 32-bit byte offset (lane * sizeof(ST) < 2^32 by validation of
// the z-plane size), so the compiler can address with a scalar 64-bit base plus a 32-bit
// vector offset instead of a 64-bit address per lane.
template <class ST>
__device__ __forceinline__ ST ldp(const ST *base, uint64_t uniform, uint32_t lane) {
  const uint32_t boff = lane * uint32_t(sizeof(ST));
  return *reinterpret_cast<const ST *>(reinterpret_cast<const unsigned char *>(base + uniform) + boff);
}
template <class ST>
__device__ __forceinline__ void stp(ST *base, uint64_t uniform, uint32_t lane, ST v) {
  const uint32_t boff = lane * uint32_t(sizeof(ST));
  __builtin_nontemporal_store(v, reinterpret_cast<ST *>(reinterpret_cast<unsigned char *>(base + uniform) + boff));
}

// natural-index helpers for the batched kernel (cell = (z * ny + y) * nx + x inside a box)
template <class ST>
__device__ __forceinline__ ST ld(const ST *base, uint32_t plane, int i, uint32_t cell) {
  return base[size_t(i) * plane + cell];
}
template <class ST>
__device__ __forceinline__ void st(ST *base, uint32_t plane, int i, uint32_t cell, ST v) {
  __builtin_nontemporal_store(v, base + size_t(i) * plane + cell);
}

template <int D>
struct NbrNat {
  uint32_t rows[3][3];
  uint32_t xs[3];
  __device__ __forceinline__ NbrNat(int x, int y, int z, int nx, int ny, int nz) {
    xs[0] = uint32_t(x == 0 ? nx - 1 : x - 1);
    xs[1] = uint32_t(x);
    xs[2] = uint32_t(x == nx - 1 ? 0 : x + 1);
    const int yy[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
    const int zz[3] = {D == 3 ? (z == 0 ? nz - 1 : z - 1) : z, z, D == 3 ? (z == nz - 1 ? 0 : z + 1) : z};
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) rows[b][c] = (uint32_t(zz[c]) * uint32_t(ny) + uint32_t(yy[b])) * uint32_t(nx);
  }
  __device__ __forceinline__ uint32_t at(int cx, int cy, int cz, int s) const {
    return rows[1 + s * cy][1 + s * cz] + xs[1 + s * cx];
  }
};

// ---------------------------------------------------------------------------------------
// fused stream + collide
// ---------------------------------------------------------------------------------------
template <int S, int SP, int EQ, bool REG, class ST, class CT, int PAT, bool FORCE = false, bool CROSS = false>
__global__ void __launch_bounds__(512) sweep_kernel(SweepArgs<ST, CT> a) {
  using L = Lat<S>;
  const CellPos p = tile_cell_args(a, 1);
  if (!p.valid) return;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz, a.L);

  CT g[L::G];
  sfor<L::G>([&](auto E) { g[E] = CT(0); });
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
    if constexpr (PAT == PULL) {
      g[L::gidx(i)] = CT(ldp(a.src, (uint64_t(i) * a.L.ps) + nb.zpart(cz, -1), nb.lane(cx, cy, -1)));
    } else if constexpr (PAT == PUSH) {
      g[L::gidx(i)] = CT(ldp(a.src, (uint64_t(i) * a.L.ps) + nb.zpart(0, 1), nb.lane(0, 0, 1)));
    } else if constexpr (PAT == AA_EVEN) {
      g[L::gidx(i)] = CT(ldp(a.src, (uint64_t(i) * a.L.ps) + nb.zpart(0, 1), nb.lane(0, 0, 1)));
    } else if constexpr (PAT == AA_ODD) {
      g[L::gidx(i)] = CT(ldp(a.src, (uint64_t(L::opp(i)) * a.L.ps) + nb.zpart(cz, -1), nb.lane(cx, cy, -1)));
    } else if constexpr (PAT == TW_EVEN || PAT == TW_ODD) {
      // Esoteric Twist: population i sits at x + (-xi)^+, slot i on even steps, opp(i) on odd
      constexpr int slot = PAT == TW_EVEN ? i : L::opp(i);
      g[L::gidx(i)] = CT(ldp(a.src, (uint64_t(slot) * a.L.ps) + nb.zpart(cz < 0, 1), nb.lane(cx < 0, cy < 0, 1)));
    } else {
      // Esoteric Pull: odd directions (and the rest) sit at the own node, their opposites at
      // x - xi; even steps find every population in the opposite slot, odd steps in its own
      constexpr int slot = PAT == ESO_EVEN ? L::opp(i) : i;
      if constexpr (i == 0 || (i & 1)) {
        g[L::gidx(i)] = CT(ldp(a.src, (uint64_t(slot) * a.L.ps) + nb.zpart(0, 1), nb.lane(0, 0, 1)));
      } else {
        g[L::gidx(i)] = CT(ldp(a.src, (uint64_t(slot) * a.L.ps) + nb.zpart(cz, -1), nb.lane(cx, cy, -1)));
      }
    }
  });

  if (a.absolute) sfor<L::Q>([&](auto I) { g[L::gidx(I)] -= CT(L::w(I)); });
  if constexpr (FORCE) {
    CT F[3] = {a.fconst[0], a.fconst[1], a.fconst[2]};
    if (a.ffield) {
      const uint64_t nc = uint64_t(a.nx) * uint64_t(a.ny) * uint64_t(a.nz);
      const uint64_t cell = (uint64_t(p.z) * uint64_t(a.ny) + uint64_t(p.y)) * uint64_t(a.nx) + uint64_t(p.x);
      F[0] += a.ffield[cell];
      F[1] += a.ffield[nc + cell];
      F[2] += a.ffield[2 * nc + cell];
    }
    if constexpr (L::D == 2) F[2] = CT(0);
    collide<S, SP, EQ, REG, CT, true, CROSS>(g, a.R, a.grav, F, a.force_model);
  } else {
    collide<S, SP, EQ, REG, CT, false, CROSS>(g, a.R, a.grav);
  }
  if (a.absolute) sfor<L::Q>([&](auto I) { g[L::gidx(I)] += CT(L::w(I)); });

  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
    const ST v = ST(g[L::gidx(i)]);
    if constexpr (PAT == PULL) {
      stp(a.dst, (uint64_t(i) * a.L.ps) + nb.zpart(0, 1), nb.lane(0, 0, 1), v);
    } else if constexpr (PAT == PUSH) {
      stp(a.dst, (uint64_t(i) * a.L.ps) + nb.zpart(cz, +1), nb.lane(cx, cy, +1), v);
    } else if constexpr (PAT == AA_EVEN) {
      stp(a.dst, (uint64_t(L::opp(i)) * a.L.ps) + nb.zpart(0, 1), nb.lane(0, 0, 1), v);
    } else if constexpr (PAT == AA_ODD) {
      stp(a.dst, (uint64_t(i) * a.L.ps) + nb.zpart(cz, +1), nb.lane(cx, cy, +1), v);
    } else if constexpr (PAT == TW_EVEN || PAT == TW_ODD) {
      // to x + (xi)^+, the home node of opp(i), in the other slot than the one read
      constexpr int slot = PAT == TW_EVEN ? L::opp(i) : i;
      stp(a.dst, (uint64_t(slot) * a.L.ps) + nb.zpart(cz > 0, 1), nb.lane(cx > 0, cy > 0, 1), v);
    } else {
      // odd directions go to x + xi, the others stay; the even step keeps the slot index,
      // the odd step writes the opposite slot (the same locations the loads read)
      constexpr int slot = PAT == ESO_EVEN ? i : L::opp(i);
      if constexpr (i != 0 && (i & 1)) {
        stp(a.dst, (uint64_t(slot) * a.L.ps) + nb.zpart(cz, +1), nb.lane(cx, cy, +1), v);
      } else {
        stp(a.dst, (uint64_t(slot) * a.L.ps) + nb.zpart(0, 1), nb.lane(0, 0, 1), v);
      }
    }
  });
}

// ---------------------------------------------------------------------------------------
// vectorised sweep: V x-adjacent cells per lane (V = 2 for FP32 and FP64, 4 for FP16: 8- or
// 16-byte accesses; wider FP32 vectors cost more registers than they gain in bandwidth)
// Requires nx % (blockDim.x * V) == 0, so every wave covers 64 V consecutive cells of one row.
// Each population row segment is read with one aligned vector load; the x - 1 and x + 1
// neighbours of the first and last cell come from the adjacent lane through a wave shift
// (DPP), and lanes 0 and 63 fetch the cell beyond their wave with one wrapped scalar load.
// ---------------------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp(int(b), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, (long long)(unsigned(lo)) | ((long long)hi << 32));
}
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane l receives lane l - 1
constexpr int DPP_WAVE_SHL1 = 0x130;  // lane l receives lane l + 1

template <class ST, int V> struct VecOf;
template <> struct VecOf<float, 2> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct VecOf<double, 2> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct VecOf<_Float16, 4> { typedef _Float16 T __attribute__((ext_vector_type(4))); };

template <class ST> struct VecWidth { static constexpr int V = sizeof(ST) == 2 ? 4 : 2; };

template <int S, int SP, int EQ, bool REG, class ST, class CT, int PAT>
__global__ void __launch_bounds__(256) sweepv_kernel(SweepArgs<ST, CT> a) {
  using L = Lat<S>;
  constexpr int V = VecWidth<ST>::V;
  using VT = typename VecOf<ST, V>::T;
  static_assert(PAT == PULL || PAT == AA_EVEN, "vectorised sweep: pull and AA even steps");
  const CellPos pc = tile_cell_args(a, V);
  const int x0 = pc.x, y = pc.y, z = pc.z;
  if (y >= a.ny) return;  // whole waves (blockDim.x is a multiple of 64)
  const Nbr<L::D> nb(x0, y, z, a.nx, a.ny, a.nz, a.L);
  const uint32_t lane_id = threadIdx.x & 63u;
  const uint32_t xw_lo = uint32_t(x0 == 0 ? a.nx - 1 : x0 - 1);       // cell before this lane
  const uint32_t xw_hi = uint32_t(x0 + V == a.nx ? 0 : x0 + V);       // cell after this lane

  CT g[V][L::G];
  sfor<V>([&](auto K) { sfor<L::G>([&](auto E) { g[K][E] = CT(0); }); });
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
    constexpr int gi = L::gidx(i);
    uint64_t uni;
    uint32_t row;
    if constexpr (PAT == PULL) {
      uni = (uint64_t(i) * a.L.ps) + nb.zpart(cz, -1);
      row = nb.yoff[1 - cy];
    } else {
      uni = (uint64_t(i) * a.L.ps) + nb.zpart(0, 1);
      row = nb.yoff[1];
    }
    const ST *rp = a.src + uni + row;
    const VT w = *reinterpret_cast<const VT *>(rp + x0);
    CT own[V];
    sfor<V>([&](auto K) { constexpr int k = decltype(K)::value; own[k] = CT(w[k]); });
    if constexpr (PAT == AA_EVEN || cx == 0) {
      sfor<V>([&](auto K) { g[K][gi] = own[K]; });
    } else if constexpr (cx == 1) {  // source x - 1
      CT prev = dpp_mov<DPP_WAVE_SHR1>(own[V - 1]);
      if (lane_id == 0) prev = CT(rp[xw_lo]);
      g[0][gi] = prev;
      sfor<V - 1>([&](auto K) { g[K + 1][gi] = own[K]; });
    } else {  // source x + 1
      CT next = dpp_mov<DPP_WAVE_SHL1>(own[0]);
      if (lane_id == 63) next = CT(rp[xw_hi]);
      sfor<V - 1>([&](auto K) { g[K][gi] = own[K + 1]; });
      g[V - 1][gi] = next;
    }
  });

  sfor<V>([&](auto K) {
    if (a.absolute) sfor<L::Q>([&](auto I) { g[K][L::gidx(I)] -= CT(L::w(I)); });
    collide<S, SP, EQ, REG, CT>(g[K], a.R, a.grav);
    if (a.absolute) sfor<L::Q>([&](auto I) { g[K][L::gidx(I)] += CT(L::w(I)); });
  });

  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int slot = PAT == PULL ? i : L::opp(i);
    VT o;
    sfor<V>([&](auto K) { constexpr int k = decltype(K)::value; o[k] = ST(g[k][L::gidx(i)]); });
    ST *dp = a.dst + ((uint64_t(slot) * a.L.ps) + nb.zpart(0, 1)) + nb.yoff[1];
    __builtin_nontemporal_store(o, reinterpret_cast<VT *>(dp + x0));
  });
}

// ---------------------------------------------------------------------------------------
// LDS-staged pull sweep: a block of TW threads owns TW consecutive cells of one row
// (x0 .. x0 + TW - 1, with nx % TW == 0).  It first copies the Q source row segments it
// gathers from, [x0 - E, x0 + TW + E) of population i in row (y - cy, z - cz), where E is the
// number of elements in one 16-byte chunk, straight from HBM into LDS with gfx950's
// global-to-LDS loads (16 bytes per lane, no register round trip; each wave's load fills
// 64 consecutive chunks of LDS), waits for them, and then every thread reads its Q values
// from LDS at x - cx, collides in registers and stores its populations like the register
// kernel.  The LDS image of the block holds Q segments of SEG = TW / E + 2 chunks each.
// ---------------------------------------------------------------------------------------
template <int S>
struct DirCode {
  // (cx + 1) | (cy + 1) << 2 | (cz + 1) << 4 of population i, ten populations per word
  static constexpr uint64_t word(int w) {
    uint64_t v = 0;
    for (int k = 0; k < 10; ++k) {
      const int i = w * 10 + k;
      if (i < Lat<S>::Q) {
        const uint64_t code = uint64_t(Lat<S>::c(i, 0) + 1) | (uint64_t(Lat<S>::c(i, 1) + 1) << 2) |
                              (uint64_t(Lat<S>::c(i, 2) + 1) << 4);
        v |= code << (6 * k);
      }
    }
    return v;
  }
  __device__ static __forceinline__ uint32_t of(uint32_t i) {
    constexpr uint64_t w0 = word(0), w1 = word(1), w2 = word(2);
    const uint32_t w = i / 10u, k = i - w * 10u;
    const uint64_t v = w == 0 ? w0 : (w == 1 ? w1 : w2);
    return uint32_t(v >> (6u * k)) & 63u;
  }
};

template <class ST, int TW>
struct StageGeom {
  static constexpr int E = 16 / int(sizeof(ST));  // elements per 16-byte chunk
  static constexpr int SEG = TW / E + 2;          // chunks per population segment
};

template <int S, class ST, int TW>
constexpr int stage_lds_bytes() {
  return Lat<S>::Q * StageGeom<ST, TW>::SEG * 16;
}

template <int S, int SP, int EQ, bool REG, class ST, class CT, int TW>
__global__ void __launch_bounds__(TW) sweepl_kernel(SweepArgs<ST, CT> a) {
  using L = Lat<S>;
  constexpr int E = StageGeom<ST, TW>::E;
  constexpr int SEG = StageGeom<ST, TW>::SEG;
  constexpr int NCH = L::Q * SEG;
  constexpr int ROUNDS = (NCH + TW - 1) / TW;
  extern __shared__ __attribute__((aligned(16))) unsigned char stage_lds[];
  const CellPos p = tile_cell_args(a, 1);  // bx == TW, by == 1: whole tiles, p.valid everywhere
  const uint32_t t = threadIdx.x;
  const uint32_t x0 = uint32_t(p.x) - t;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz, a.L);
  const uint32_t xl = x0 == 0 ? uint32_t(a.nx - E) : x0 - E;            // left chunk (wrapped)
  const uint32_t xr = x0 + TW == uint32_t(a.nx) ? 0u : x0 + TW;          // right chunk (wrapped)
  const uint32_t wave_chunk0 = (t & ~63u);
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const uint32_t cw = uint32_t(r * TW) + wave_chunk0;  // first chunk of this wave's load
    if (cw >= uint32_t(NCH)) break;                      // wave-uniform
    const uint32_t c = cw + (t & 63u);
    if (c < uint32_t(NCH)) {
      const uint32_t i = c / uint32_t(SEG), k = c - i * uint32_t(SEG);
      const uint32_t code = DirCode<S>::of(i);
      const int cx = int(code & 3u) - 1, cy = int((code >> 2) & 3u) - 1, cz = int((code >> 4) & 3u) - 1;
      (void)cx;
      const uint32_t xe = k == 0 ? xl : (k == uint32_t(SEG - 1) ? xr : x0 + (k - 1) * uint32_t(E));
      const ST *g = a.src + (uint64_t(i) * a.L.ps + nb.zpart(cz, -1)) + (nb.yoff[1 - cy] + xe);
      // address-space conversions (flat -> global, flat -> LDS) need C-style casts
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(g),
                                       (__attribute__((address_space(3))) void *)(stage_lds + size_t(cw) * 16u),
                                       16, 0, 0);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  const ST *ls = reinterpret_cast<const ST *>(stage_lds);
  CT g[L::G];
  sfor<L::G>([&](auto K) { g[K] = CT(0); });
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::c(i, 0);
    g[L::gidx(i)] = CT(ls[i * SEG * E + E - cx + int(t)]);
  });
  if (a.absolute) sfor<L::Q>([&](auto I) { g[L::gidx(I)] -= CT(L::w(I)); });
  collide<S, SP, EQ, REG, CT>(g, a.R, a.grav);
  if (a.absolute) sfor<L::Q>([&](auto I) { g[L::gidx(I)] += CT(L::w(I)); });
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    stp(a.dst, (uint64_t(i) * a.L.ps) + nb.zpart(0, 1), nb.lane(0, 0, 1), ST(g[L::gidx(i)]));
  });
}

// ---------------------------------------------------------------------------------------
// AA odd step with LDS-shifted stores.  The odd step writes slot i at x + xi, one element off
// the row alignment for cx != 0, so every wave of the per-cell kernel writes two partial
// cache lines per shifted population.  Here a block (bx x by threads, whole tiles along x,
// nx % bx == 0) first puts the post-collision values of its shifted populations into LDS,
// then each thread stores position x0 + tx of a row segment with the value of cell
// x0 + tx - cx, so the block writes whole lines except at its two ends: position x0 (cx = +1)
// or x0 + bx - 1 (cx = -1) is left to the neighbouring block, and the edge thread stores its
// own value beyond the block at x0 + bx or x0 - 1 (wrapped).  Every location is still read
// and written by the block of the cell that owns it (reads before the barrier, writes after),
// so the in-place step stays race-free.
// ---------------------------------------------------------------------------------------
template <int S>
constexpr int n_shifted() {
  int n = 0;
  for (int i = 0; i < Lat<S>::Q; ++i) n += Lat<S>::c(i, 0) != 0;
  return n;
}
template <int S>
constexpr int shifted_index(int i) {  // rank of population i among those with cx != 0
  int n = 0;
  for (int j = 0; j < i; ++j) n += Lat<S>::c(j, 0) != 0;
  return n;
}

template <int S, int SP, int EQ, bool REG, class ST, class CT>
__global__ void __launch_bounds__(256) sweep_aa_odd_shift_kernel(SweepArgs<ST, CT> a) {
  using L = Lat<S>;
  extern __shared__ __attribute__((aligned(16))) unsigned char shift_lds[];
  ST *sh = reinterpret_cast<ST *>(shift_lds);  // [n_shifted][by][bx]
  const CellPos p = tile_cell_args(a, 1);      // p.x < nx always (whole tiles along x)
  const int bx = a.bx, nthreads = a.bx * a.by;
  const int tx = int(threadIdx.x), tid = int(threadIdx.y) * bx + tx;
  const Nbr<L::D> nb(p.x, p.valid ? p.y : 0, p.z, a.nx, a.ny, a.nz, a.L);
  CT g[L::G];
  sfor<L::G>([&](auto E) { g[E] = CT(0); });
  if (p.valid) {
    sfor<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
      g[L::gidx(i)] = CT(ldp(a.src, (uint64_t(L::opp(i)) * a.L.ps) + nb.zpart(cz, -1), nb.lane(cx, cy, -1)));
    });
    if (a.absolute) sfor<L::Q>([&](auto I) { g[L::gidx(I)] -= CT(L::w(I)); });
    collide<S, SP, EQ, REG, CT>(g, a.R, a.grav);
    if (a.absolute) sfor<L::Q>([&](auto I) { g[L::gidx(I)] += CT(L::w(I)); });
  }
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
    const ST v = ST(g[L::gidx(i)]);
    if constexpr (cx == 0) {
      if (p.valid) stp(a.dst, (uint64_t(i) * a.L.ps) + nb.zpart(cz, +1), nb.lane(0, cy, +1), v);
    } else {
      sh[shifted_index<S>(i) * nthreads + tid] = v;
    }
  });
  __syncthreads();
  if (!p.valid) return;
  const uint32_t xo = uint32_t(p.x);
  const uint32_t x_lo = xo == 0 ? uint32_t(a.nx - 1) : xo - 1;          // x - 1, wrapped
  const uint32_t x_hi = xo + 1 == uint32_t(a.nx) ? 0u : xo + 1;          // x + 1, wrapped
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
    if constexpr (cx != 0) {
      const uint64_t uni = (uint64_t(i) * a.L.ps) + nb.zpart(cz, +1);
      const uint32_t row = nb.yoff[1 + cy];
      const ST *shi = sh + shifted_index<S>(i) * nthreads + (tid - tx);
      const int src_tx = tx - cx;  // the cell whose value lands on this thread's position
      if (src_tx >= 0 && src_tx < bx) stp(a.dst, uni, row + xo, shi[src_tx]);
      // the edge value that leaves the block
      if (cx == 1 && tx == bx - 1) stp(a.dst, uni, row + x_hi, shi[tx]);
      if (cx == -1 && tx == 0) stp(a.dst, uni, row + x_lo, shi[tx]);
    }
  });
}

// ---------------------------------------------------------------------------------------
// readers / writers of the canonical state
// ---------------------------------------------------------------------------------------
struct FieldArgs {
  void *buf;          // population buffer (storage type), first element of the box
  Strides L;          // storage layout of the buffer
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
  int absolute;           // nonzero: buffers hold absolute populations f = df + w
  int forced;             // nonzero: velocities are Guo's (j + F/2) / rho
  const void *ffield;     // body force per cell [3][ncells] (double if ffield_f64, else float) or null
  int ffield_f64;
  double fconst[3];       // constant body force
};

// storage address (uniform part, lane part) of the canonical df_i(x) for layout GM
template <int S, int GM>
__device__ __forceinline__ void canon_addr(const Nbr<Lat<S>::D> &nb, const Strides &L, int i, int cx, int cy,
                                           int cz, uint64_t &uni, uint32_t &lane) {
  if constexpr (GM == G_NATURAL) {
    uni = uint64_t(i) * L.ps + nb.zpart(0, 1);
    lane = nb.lane(0, 0, 1);
  } else if constexpr (GM == G_SHIFTED) {
    uni = uint64_t(i) * L.ps + nb.zpart(cz, -1);
    lane = nb.lane(cx, cy, -1);
  } else if constexpr (GM == G_AA_ODD) {
    uni = uint64_t(Lat<S>::opp(i)) * L.ps + nb.zpart(cz, -1);
    lane = nb.lane(cx, cy, -1);
  } else if constexpr (GM == G_TW_EVEN || GM == G_TW_ODD) {
    // Esoteric Twist: slot i (even times) or opp(i) (odd times) at x + (-xi)^+
    uni = uint64_t(GM == G_TW_EVEN ? i : Lat<S>::opp(i)) * L.ps + nb.zpart(cz < 0, 1);
    lane = nb.lane(cx < 0, cy < 0, 1);
  } else {
    // Esoteric Pull: slot opp(i) (even times) or i (odd times); odd i at the own node,
    // even i > 0 at x - xi
    const int slot = GM == G_ESO_EVEN ? Lat<S>::opp(i) : i;
    if (i == 0 || (i & 1)) {
      uni = uint64_t(slot) * L.ps + nb.zpart(0, 1);
      lane = nb.lane(0, 0, 1);
    } else {
      uni = uint64_t(slot) * L.ps + nb.zpart(cz, -1);
      lane = nb.lane(cx, cy, -1);
    }
  }
}

__device__ __forceinline__ uint32_t nat_cell(const FieldArgs &a, const CellPos &p) {
  return (uint32_t(p.z) * uint32_t(a.ny) + uint32_t(p.y)) * uint32_t(a.nx) + uint32_t(p.x);
}

template <int S, int GM, class ST>
__device__ __forceinline__ void gather_canon(const FieldArgs &a, const CellPos &p, double *f) {
  using L = Lat<S>;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz, a.L);
  const ST *buf = static_cast<const ST *>(a.buf);
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    uint64_t uni;
    uint32_t lane;
    canon_addr<S, GM>(nb, a.L, i, L::c(i, 0), L::c(i, 1), L::c(i, 2), uni, lane);
    f[i] = double(ldp(buf, uni, lane)) - (a.absolute ? L::w(i) : 0.0);
  });
}

// df(0) = f_eq(rho, u) - f0, written in layout GM (G_SHIFTED for pull, G_NATURAL for AA,
// G_ESO_EVEN for Esoteric Pull, G_TW_EVEN for Esoteric Twist)
template <int S, int SP, int EQ, int GM, class ST>
__global__ void __launch_bounds__(256) init_kernel(FieldArgs a) {
  using L = Lat<S>;
  const CellPos p = tile_cell(a.nx, a.ny, a.tiles_x, a.tiles_y, 0);
  if (!p.valid) return;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz, a.L);
  const uint32_t self = nat_cell(a, p);
  const double drho = a.rho_in[self] - 1.0;
  double u[3] = {a.u_in[self], a.u_in[size_t(a.ncells) + self], L::D == 3 ? a.u_in[2 * size_t(a.ncells) + self] : 0.0};
  double g[L::G];
  equilibrium_dev<S, SP, EQ, double>(g, drho, u, a.grav);
  ST *buf = static_cast<ST *>(a.buf);
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    uint64_t uni;
    uint32_t lane;
    canon_addr<S, GM>(nb, a.L, i, L::c(i, 0), L::c(i, 1), L::c(i, 2), uni, lane);
    stp(buf, uni, lane, ST(g[L::gidx(i)] + (a.absolute ? L::w(i) : 0.0)));
  });
}

template <int S, int GM, class ST>
__global__ void __launch_bounds__(256) export_kernel(FieldArgs a) {
  using L = Lat<S>;
  const CellPos p = tile_cell(a.nx, a.ny, a.tiles_x, a.tiles_y, 0);
  if (!p.valid) return;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz, a.L);
  const uint32_t self = nat_cell(a, p);
  const ST *buf = static_cast<const ST *>(a.buf);
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if (i >= a.i0 && i < a.i1) {
      uint64_t uni;
      uint32_t lane;
      canon_addr<S, GM>(nb, a.L, i, L::c(i, 0), L::c(i, 1), L::c(i, 2), uni, lane);
      a.pop[size_t(i - a.i0) * a.ncells + self] = double(ldp(buf, uni, lane)) - (a.absolute ? L::w(i) : 0.0);
    }
  });
}

template <int S, int GM, class ST>
__global__ void __launch_bounds__(256) import_kernel(FieldArgs a) {
  using L = Lat<S>;
  const CellPos p = tile_cell(a.nx, a.ny, a.tiles_x, a.tiles_y, 0);
  if (!p.valid) return;
  const Nbr<L::D> nb(p.x, p.y, p.z, a.nx, a.ny, a.nz, a.L);
  const uint32_t self = nat_cell(a, p);
  ST *buf = static_cast<ST *>(a.buf);
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if (i >= a.i0 && i < a.i1) {
      uint64_t uni;
      uint32_t lane;
      canon_addr<S, GM>(nb, a.L, i, L::c(i, 0), L::c(i, 1), L::c(i, 2), uni, lane);
      stp(buf, uni, lane, ST(a.pop[size_t(i - a.i0) * a.ncells + self] + (a.absolute ? L::w(i) : 0.0)));
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
  const uint32_t self = nat_cell(a, p);
  if (a.forced) {
    sfor<3>([&](auto Dd) {
      constexpr int d = decltype(Dd)::value;
      double F = a.fconst[d];
      if (a.ffield) {
        const size_t k = size_t(d) * a.ncells + self;
        F += a.ffield_f64 ? static_cast<const double *>(a.ffield)[k] : double(static_cast<const float *>(a.ffield)[k]);
      }
      if (L::D == 3 || d < 2) j[d] += 0.5 * F;
    });
  }
  a.rho_out[self] = rho;
  a.u_out[self] = j[0] / rho;
  a.u_out[size_t(a.ncells) + self] = j[1] / rho;
  a.u_out[2 * size_t(a.ncells) + self] = j[2] / rho;
}

// grid-stride over cells in a fixed order per thread, block tree in LDS -> deterministic
constexpr int DIAG_THREADS = 256;

// Sum of v over the 64 lanes of a wave by a butterfly of lane exchanges (the lanes pair up
// at distances 32, 16, ..., 1); every lane ends with the total.  The order of the additions
// is fixed, so the result is reproducible bit for bit.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Six block-wide sums of DIAG_THREADS threads: wave sums first, then the DIAG_THREADS / 64
// wave totals in wave order; red[k][0] holds sum k afterwards (fixed order, deterministic).
__device__ __forceinline__ void block_sum6(const double acc[6], double (*red)[DIAG_THREADS / 64]) {
  const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double w = wave_sum(acc[k]);
    if (lane == 0) red[k][wave] = w;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0.0;
    for (int w = 0; w < DIAG_THREADS / 64; ++w) t += red[threadIdx.x][w];
    red[threadIdx.x][0] = t;
  }
  __syncthreads();
}
template <int S, int GM, class ST>
__global__ void __launch_bounds__(DIAG_THREADS) diag_kernel(FieldArgs a) {
  using L = Lat<S>;
  __shared__ double red[6][DIAG_THREADS / 64];
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
  block_sum6(acc, red);
  if (threadIdx.x < 6) a.partials[size_t(blockIdx.x) * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// final fixed-order sum of nblocks x 6 partials by one block
__global__ void __launch_bounds__(DIAG_THREADS) diag_final_kernel(const double *partials, int nblocks, double *out);

}  // namespace lbm
