// Batched ensemble sweep: many independent periodic boxes, one launch per time step.
//
// Populations of all boxes share one SoA buffer, plane stride ntot = sum of box cells; box b
// occupies cells [off_b, off_b + ncells_b) of every plane.  Blocks walk a flat tile list:
// tile k belongs to box tile_box[k] and covers blockDim.x consecutive cells of that box in
// memory order (x fastest; the tile size is a launch parameter, chosen by the autotuner), so
// every block reads and writes contiguous rows whatever the box edge.  Blocks
// take tiles in XCD order (each XCD a contiguous range), so the cache lines that neighbouring
// tiles share are fetched into one L2.  Two grid forms: one block per tile, or a persistent
// grid of as many blocks as fit on the chip at once, each striding over the tile list (the
// stride is a multiple of 8, so a block keeps to its XCD's range in XCD order).
#pragma once

#include "lbm_kernels.hpp"

namespace lbm {

struct BoxInfo {
  uint32_t off;     // first cell of the box in the shared planes
  uint32_t ncells;
  uint32_t tile0;   // first tile of the box
  int nx, ny, nz;
};

template <class ST, class CT>
struct BatchArgs {
  const ST *src;
  ST *dst;
  uint32_t ntot;             // plane stride
  const BoxInfo *boxes;
  const uint32_t *tile_box;  // box of every tile
  const Relax<CT> *relax;    // per-box relaxation blocks
  int swizzle;               // nonzero: consecutive tiles on one XCD (shared boundary lines in one L2)
  uint32_t ntiles;           // tiles in the list (the persistent form's loop bound)
};

constexpr int BATCH_THREADS = 256;      // default tile size (cells = threads per block)
constexpr int BATCH_MAX_THREADS = 512;

template <int S, int SP, int EQ, bool REG, class ST, class CT>
__device__ __forceinline__ void batch_tile(const BatchArgs<ST, CT> &a, uint32_t tile) {
  using L = Lat<S>;
  const uint32_t b = a.tile_box[tile];
  const BoxInfo B = a.boxes[b];
  const uint32_t c = (tile - B.tile0) * blockDim.x + threadIdx.x;
  if (c >= B.ncells) return;
  const uint32_t nxy = uint32_t(B.nx) * uint32_t(B.ny);
  const int z = int(c / nxy);
  const uint32_t r = c - uint32_t(z) * nxy;
  const int y = int(r / uint32_t(B.nx));
  const int x = int(r - uint32_t(y) * uint32_t(B.nx));
  const NbrNat<L::D> nb(x, y, z, B.nx, B.ny, B.nz);
  const ST *src = a.src + B.off;
  ST *dst = a.dst + B.off;

  CT g[L::G];
  sfor<L::G>([&](auto E) { g[E] = CT(0); });
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    g[L::gidx(i)] = CT(ld(src, a.ntot, i, nb.at(L::c(i, 0), L::c(i, 1), L::c(i, 2), -1)));
  });
  collide<S, SP, EQ, REG, CT>(g, a.relax[b], CT(0));
  sfor<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    st(dst, a.ntot, i, c, ST(g[L::gidx(i)]));
  });
}

template <int S, int SP, int EQ, bool REG, class ST, class CT, bool PERSIST = false>
__global__ void __launch_bounds__(BATCH_MAX_THREADS) batch_sweep_kernel(BatchArgs<ST, CT> a) {
  if constexpr (!PERSIST) {
    batch_tile<S, SP, EQ, REG>(a, a.swizzle ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x);
  } else {
    // the loop index k runs on XCD k % 8 (gridDim.x % 8 == 0), the XCD that xcd_tile assigns it to
    for (uint32_t k = blockIdx.x; k < a.ntiles; k += gridDim.x)
      batch_tile<S, SP, EQ, REG>(a, a.swizzle ? xcd_tile(k, a.ntiles) : k);
  }
}

template <int S, int STORE>
struct BTable {
  static const void *sweep(int sp, int reg, bool persistent);
};

const void *batch_sweep_fn(int s, int store, int sp, int reg, bool persistent);

}  // namespace lbm
