// Runtime of the lattice Boltzmann library: contexts, launches, hipGraph replay of time
// loops, readers/writers of the canonical state, reductions, launch-shape autotuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_dispatch.hpp"
#include "lbm_kernels.hpp"
#include "lbm_literal.hpp"
#include "lbm_method.hpp"

static_assert(lbm::kSpaceSrt == lbm::SRT, "SRT space id");
static_assert(lbm::kLitA == lbm::LIT_A && lbm::kLitB == lbm::LIT_B && lbm::kLitC == lbm::LIT_C, "literal form ids");

namespace lbm {

// ---------------------------------------------------------------------------------------
// dispatch over the per-(stencil, storage) tables
// ---------------------------------------------------------------------------------------
#define LBM_TABLE_CALL(FN, ...)                                                   \
  switch (s * 3 + store) {                                                        \
    case 0: return KTable<D2Q9, F64>::FN(__VA_ARGS__);                            \
    case 1: return KTable<D2Q9, F32>::FN(__VA_ARGS__);                            \
    case 2: return KTable<D2Q9, F16>::FN(__VA_ARGS__);                            \
    case 3: return KTable<D3Q19, F64>::FN(__VA_ARGS__);                           \
    case 4: return KTable<D3Q19, F32>::FN(__VA_ARGS__);                           \
    case 5: return KTable<D3Q19, F16>::FN(__VA_ARGS__);                           \
    case 6: return KTable<D3Q27, F64>::FN(__VA_ARGS__);                           \
    case 7: return KTable<D3Q27, F32>::FN(__VA_ARGS__);                           \
    case 8: return KTable<D3Q27, F16>::FN(__VA_ARGS__);                           \
    case 9: return KTable<D3Q15, F64>::FN(__VA_ARGS__);                           \
    case 10: return KTable<D3Q15, F32>::FN(__VA_ARGS__);                          \
    case 11: return KTable<D3Q15, F16>::FN(__VA_ARGS__);                          \
  }                                                                               \
  return nullptr;

const void *sweep_fn(int s, int store, int sp, int eq, int reg, int pat) { LBM_TABLE_CALL(sweep, sp, eq, reg, pat) }
const void *sweepv_fn(int s, int store, int sp, int eq, int reg, int pat) { LBM_TABLE_CALL(sweepv, sp, eq, reg, pat) }
const void *sweepl_fn(int s, int store, int sp, int eq, int reg, int tw) { LBM_TABLE_CALL(sweepl, sp, eq, reg, tw) }
// LDS image of sweepl_kernel: Q segments of StageGeom<ST, TW>::SEG 16-byte chunks
int sweepl_lds_bytes(int s, int store, int tw) {
  const int q = s == D2Q9 ? 9 : (s == D3Q19 ? 19 : (s == D3Q15 ? 15 : 27));
  const int e = store == F64 ? 2 : (store == F32 ? 4 : 8);
  return q * (tw / e + 2) * 16;
}
const void *sweep_aa_shift_fn(int s, int store, int sp, int eq, int reg) { LBM_TABLE_CALL(sweep_aa_shift, sp, eq, reg) }
static_assert(stage_lds_bytes<D3Q27, float, 256>() == 27 * (256 / 4 + 2) * 16, "staged LDS image");
static_assert(stage_lds_bytes<D3Q19, double, 128>() == 19 * (128 / 2 + 2) * 16, "staged LDS image");
const void *sweep_mfma_fn(int s, int store, int sp, int reg) { LBM_TABLE_CALL(sweep_mfma, sp, reg) }
const void *sweep_literal_fn(int s, int store, int sp, int form) { LBM_TABLE_CALL(sweep_literal, sp, form) }
const void *sweep_literal_cross_fn(int s, int store, int form) { LBM_TABLE_CALL(sweep_literal_cross, form) }
const void *sweep_force_fn(int s, int store, int sp, int pat) { LBM_TABLE_CALL(sweep_force, sp, pat) }
const void *sweep_cross_fn(int s, int store, int pat) { LBM_TABLE_CALL(sweep_cross, pat) }
const void *sweep_force_cross_fn(int s, int store, int pat) { LBM_TABLE_CALL(sweep_force_cross, pat) }
const void *init_fn(int s, int store, int sp, int eq, int gm) { LBM_TABLE_CALL(init, sp, eq, gm) }
const void *export_fn(int s, int store, int gm) { LBM_TABLE_CALL(exporter, gm) }
const void *import_fn(int s, int store, int gm) { LBM_TABLE_CALL(importer, gm) }
const void *macro_fn(int s, int store, int gm) { LBM_TABLE_CALL(macro, gm) }
const void *diag_fn(int s, int store, int gm) { LBM_TABLE_CALL(diag, gm) }

__global__ void __launch_bounds__(DIAG_THREADS) diag_final_kernel(const double *partials, int nblocks, double *out) {
  __shared__ double red[6][DIAG_THREADS / 64];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += DIAG_THREADS)
    for (int k = 0; k < 6; ++k) acc[k] += partials[size_t(b) * 6 + k];
  block_sum6(acc, red);
  if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

// plain copy, one 16-byte vector per lane and one lane per vector: the practical HBM ceiling
// (the fastest of the copy forms measured on MI355X; grid-stride and unrolled forms were slower)
typedef unsigned int lbm_v4u __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) copy_kernel(lbm_v4u *__restrict__ dst, const lbm_v4u *__restrict__ src, size_t n) {
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(src[i], dst + i);
}

const void *diag_final_fn() { return reinterpret_cast<const void *>(&diag_final_kernel); }
const void *copy_fn() { return reinterpret_cast<const void *>(&copy_kernel); }

static lbm_status hip_fail(hipError_t e, const char *what) {
  return fail(LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHECK(call, what)                 \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Population buffers larger than the free device memory are refused with LBM_ENOMEM before
// hipMalloc is asked for them: an allocation beyond the device's memory is reported by the HIP
// runtime as a missing device and leaves the process unable to create streams afterwards.
static lbm_status check_free_memory(size_t need, const char *what) {
  size_t free_b = 0, total_b = 0;
  const hipError_t e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) return hip_fail(e, "device memory query");
  if (need > free_b)
    return fail(LBM_ENOMEM, std::string(what) + " allocation needs " + std::to_string(need) + " bytes, " +
                                std::to_string(free_b) + " of " + std::to_string(total_b) +
                                " bytes of device memory are free");
  return LBM_OK;
}

static bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Two HIP events released on every return path of the timing helpers.
struct EventPair {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EventPair() = default;
  EventPair(const EventPair &) = delete;
  EventPair &operator=(const EventPair &) = delete;
  ~EventPair() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  hipError_t create() {
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    return e;
  }
  // elapsed milliseconds between e0 and e1 (after waiting for e1)
  hipError_t elapsed(float *ms) {
    hipError_t e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    return e;
  }
};

}  // namespace lbm

using namespace lbm;

struct lbm_ctx {
  lbm_params p;
  std::vector<double> omegas;
  int s = 0, q = 0, d = 0, space = 0, eq = 0, store = 0, pattern = 0;
  int nx = 1, ny = 1, nz = 1;
  uint32_t ncells = 0;
  Strides L{};          // storage layout strides (elements)
  int layout = 0;
  size_t elem = 4;
  RelaxHost R{};
  bool reg = false;
  void *buf[2] = {nullptr, nullptr};
  bool own[2] = {false, false};
  int nbuf = 2;
  size_t buf_bytes = 0;
  int cur = 0;        // pull: buffer holding the state
  int64_t t = 0;      // steps since init
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int bx = 64, by = 4, swz = 0;
  bool vec = false;   // vectorised sweep (V cells per lane) where the shape allows it
  bool stage = false; // LDS-staged pull sweep where the shape allows it
  int lds = 0;        // dynamic LDS reserved per sweep block: caps resident blocks per CU
  int transform = 0;  // LBM_TRANSFORM_CHIMERA or LBM_TRANSFORM_DENSE_MFMA (ablation)
  bool literal = false;  // LBM_ARITH_LITERAL: the collision form evaluated as written
  int form = 0;          // its form (kLitA / kLitB / kLitC)
  void *ffield = nullptr;  // body force per cell [3][ncells] in the compute precision, or null
  bool graphs = true;
  std::map<std::pair<int64_t, int>, hipGraphExec_t> gcache;
  double *staging = nullptr;
  size_t staging_doubles = 0;
  double *partials = nullptr;
  int diag_blocks = 0;
  int device = 0;     // the device that was current at lbm_create
  // block -> tile tables of the sweep for the current launch shape (index 1: vectorised);
  // tile_key is the (bx, by, swz) they were built for
  uint2 *tiles[2] = {nullptr, nullptr};
  int tile_key[3] = {0, 0, -1};
};

namespace lbm {

static int vec_width(int store) { return store == F16 ? 4 : 2; }
// the vectorised kernel runs when every wave covers whole 64 V-cell chunks of one row
static bool vec_ok(const lbm_ctx *c, int bx) { return bx % 64 == 0 && c->nx % (bx * vec_width(c->store)) == 0; }

// Host copy of the device's XCD order: 8 XCDs take workgroups round-robin, so block b runs
// on XCD b % 8; give each XCD a contiguous range of tiles (its own part of the box in L2).
static uint32_t xcd_tile_host(uint32_t b, uint32_t n) {
  const uint32_t per = n / 8u, rem = n % 8u;
  const uint32_t xcd = b % 8u, local = b / 8u;
  return xcd < rem ? xcd * (per + 1u) + local : rem * (per + 1u) + (xcd - rem) * per + local;
}

// populations with cx != 0 (the ones the AA odd step writes one element off the alignment)
static int n_shifted_pops(int s) {
  switch (s) {
    case D2Q9: return n_shifted<D2Q9>();
    case D3Q19: return n_shifted<D3Q19>();
    case D3Q15: return n_shifted<D3Q15>();
  }
  return n_shifted<D3Q27>();
}
static int aa_shift_lds_bytes(const lbm_ctx *c, int bx, int by) {
  return n_shifted_pops(c->s) * bx * by * int(c->elem);
}

// The LDS variant of the pattern: pull -> the LDS-staged sweep (one row of 128 or 256 cells
// per block, whole tiles along x, 16-byte aligned rows for the 16-byte global-to-LDS loads);
// AA -> the odd step with LDS-shifted stores (at most 256 threads, whole tiles along x).
static bool stage_ok(const lbm_ctx *c, int bx, int by) {
  if (c->pattern == LBM_STREAM_AA)
    return bx * by <= 256 && c->nx % bx == 0 && aa_shift_lds_bytes(c, bx, by) <= 65536;
  if (c->pattern != LBM_STREAM_PULL) return false;
  if (by != 1 || (bx != 128 && bx != 256) || c->nx % bx != 0) return false;
  for (int k = 0; k < c->nbuf; ++k)
    if (reinterpret_cast<uintptr_t>(c->buf[k]) % 16 != 0) return false;
  return (c->L.ps * c->elem) % 16 == 0 && (c->L.zs * c->elem) % 16 == 0 && (uint64_t(c->L.ys) * c->elem) % 16 == 0;
}

static bool forced(const lbm_ctx *c) {
  return c->ffield || c->p.force[0] != 0.0 || c->p.force[1] != 0.0 || c->p.force[2] != 0.0;
}

static void free_tiles(lbm_ctx *c) {
  for (int v = 0; v < 2; ++v) {
    if (c->tiles[v]) (void)hipFree(c->tiles[v]);
    c->tiles[v] = nullptr;
  }
  c->tile_key[2] = -1;
}

static const uint64_t MAX_TILE_TABLE = uint64_t(1) << 24;  // blocks; larger grids divide on the device

// Build the block -> (tx, ty, tz) tables for the current launch shape, so the sweep reads its
// tile with one scalar load instead of two integer divisions per block.  Called outside graph
// capture (it allocates); a grid without a table falls back to the division path.
static lbm_status ensure_tiles(lbm_ctx *c) {
  if (c->tile_key[0] == c->bx && c->tile_key[1] == c->by && c->tile_key[2] == c->swz) return LBM_OK;
  free_tiles(c);
  const char *env = std::getenv("LBM_TILE_TABLE");
  const bool use_table = !(env && env[0] == '0');
  for (int v = 0; v < 2 && use_table; ++v) {
    if (v == 1 && !vec_ok(c, c->bx)) continue;
    const int cells_x = c->bx * (v ? vec_width(c->store) : 1);
    const uint64_t tx = (uint64_t(c->nx) + cells_x - 1) / cells_x, ty = (uint64_t(c->ny) + c->by - 1) / c->by;
    const uint64_t n = tx * ty * uint64_t(c->nz);
    if (tx >= 65536 || ty >= 65536 || n > MAX_TILE_TABLE) continue;
    std::vector<uint2> h(n);
    for (uint64_t b = 0; b < n; ++b) {
      const uint64_t tile = c->swz ? xcd_tile_host(uint32_t(b), uint32_t(n)) : b;
      const uint64_t z = tile / (tx * ty), r = tile - z * tx * ty, y = r / tx, x = r - y * tx;
      h[b] = make_uint2(uint32_t(x | (y << 16)), uint32_t(z));
    }
    hipError_t e = hipMalloc(&c->tiles[v], n * sizeof(uint2));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      c->tiles[v] = nullptr;
      continue;  // no table: the kernel divides
    }
    HIPCHECK(hipMemcpy(c->tiles[v], h.data(), n * sizeof(uint2), hipMemcpyHostToDevice), "tile table copy");
  }
  c->tile_key[0] = c->bx;
  c->tile_key[1] = c->by;
  c->tile_key[2] = c->swz;
  return LBM_OK;
}

template <class ST, class CT>
static SweepArgs<ST, CT> make_sweep_args(const lbm_ctx *c, const void *src, void *dst, bool vec) {
  SweepArgs<ST, CT> a;
  std::memset(&a, 0, sizeof(a));
  a.src = static_cast<const ST *>(src);
  a.dst = static_cast<ST *>(dst);
  a.nx = c->nx;
  a.ny = c->ny;
  a.nz = c->nz;
  a.L = c->L;
  const int cells_x = c->bx * (vec ? vec_width(c->store) : 1);
  a.tiles_x = (c->nx + cells_x - 1) / cells_x;
  a.tiles_y = (c->ny + c->by - 1) / c->by;
  a.swizzle = c->swz;
  a.absolute = c->p.zero_centered ? 0 : 1;
  a.bx = c->bx;
  a.by = c->by;
  const bool table_ok = c->tile_key[0] == c->bx && c->tile_key[1] == c->by && c->tile_key[2] == c->swz;
  a.tile_table = table_ok ? c->tiles[vec ? 1 : 0] : nullptr;
  a.grav = CT(c->p.gravity);
  a.ffield = static_cast<const CT *>(c->ffield);
  for (int d = 0; d < 3; ++d) a.fconst[d] = CT(c->p.force[d]);
  a.force_model = c->p.force_model == LBM_FORCE_HE ? FORCE_HE : FORCE_GUO;
  for (int j = 0; j < 6; ++j)
    for (int k = 0; k < 6; ++k) a.R.b2[j][k] = CT(c->R.b2[j][k]);
  for (int j = 0; j < 7; ++j)
    for (int k = 0; k < 7; ++k) a.R.b3[j][k] = CT(c->R.b3[j][k]);
  for (int j = 0; j < 6; ++j)
    for (int k = 0; k < 6; ++k) a.R.b4[j][k] = CT(c->R.b4[j][k]);
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) a.R.b5[j][k] = CT(c->R.b5[j][k]);
  a.R.b6 = CT(c->R.b6);
  for (int j = 0; j < 7; ++j)
    for (int k = 0; k < 3; ++k) a.R.c31[j][k] = CT(c->R.c31[j][k]);
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) a.R.c51[j][k] = CT(c->R.c51[j][k]);
  for (int j = 0; j < 6; ++j)
    for (int k = 0; k < 6; ++k) a.R.c42[j][k] = CT(c->R.c42[j][k]);
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 7; ++k) a.R.c53[j][k] = CT(c->R.c53[j][k]);
  for (int k = 0; k < 6; ++k) {
    a.R.c62[k] = CT(c->R.c62[k]);
    a.R.c64[k] = CT(c->R.c64[k]);
  }
  return a;
}

template <class ST, class CT>
static hipError_t launch_sweep_t(const lbm_ctx *c, const void *fn, const void *src, void *dst, bool vec) {
  SweepArgs<ST, CT> a = make_sweep_args<ST, CT>(c, src, dst, vec);
  void *args[] = {&a};
  const dim3 grid(unsigned(uint64_t(a.tiles_x) * uint64_t(a.tiles_y) * uint64_t(c->nz)));
  return hipLaunchKernel(fn, grid, dim3(c->bx, c->by), args, size_t(c->lds), c->stream);
}

// MFMA ablation: per-wave LDS of 27 x 65 compute values (F64: doubles, else floats)
static int mfma_lds_bytes(const lbm_ctx *c) {
  const int waves = (c->bx * c->by + 63) / 64;
  return waves * 27 * 65 * (c->store == F64 ? 8 : 4);
}

template <class ST, class CT>
static hipError_t launch_sweep_lds_t(const lbm_ctx *c, const void *fn, const void *src, void *dst, int lds) {
  SweepArgs<ST, CT> a = make_sweep_args<ST, CT>(c, src, dst, false);
  void *args[] = {&a};
  const dim3 grid(unsigned(uint64_t(a.tiles_x) * uint64_t(a.tiles_y) * uint64_t(c->nz)));
  return hipLaunchKernel(fn, grid, dim3(c->bx, c->by), args, size_t(lds), c->stream);
}

static hipError_t launch_sweep_lds(const lbm_ctx *c, const void *fn, const void *src, void *dst, int lds) {
  switch (c->store) {
    case F64: return launch_sweep_lds_t<double, double>(c, fn, src, dst, lds);
    case F32: return launch_sweep_lds_t<float, float>(c, fn, src, dst, lds);
    default: return launch_sweep_lds_t<_Float16, float>(c, fn, src, dst, lds);
  }
}

static hipError_t launch_sweep(const lbm_ctx *c, const void *fn, const void *src, void *dst, bool vec) {
  switch (c->store) {
    case F64: return launch_sweep_t<double, double>(c, fn, src, dst, vec);
    case F32: return launch_sweep_t<float, float>(c, fn, src, dst, vec);
    default: return launch_sweep_t<_Float16, float>(c, fn, src, dst, vec);
  }
}

// pull and push alternate between two buffers; the other patterns run in place in one
static bool two_buffers(const lbm_ctx *c) {
  return c->pattern == LBM_STREAM_PULL || c->pattern == LBM_STREAM_PUSH;
}

// sweep kernel pattern of the step that starts at time t, and the layout of df(t)
static int step_pattern(const lbm_ctx *c, int64_t t) {
  const bool even = t % 2 == 0;
  switch (c->pattern) {
    case LBM_STREAM_PUSH: return PUSH;
    case LBM_STREAM_AA: return even ? AA_EVEN : AA_ODD;
    case LBM_STREAM_ESOTERIC_PULL: return even ? ESO_EVEN : ESO_ODD;
    case LBM_STREAM_ESOTERIC_TWIST: return even ? TW_EVEN : TW_ODD;
  }
  return PULL;
}
static int gather_mode_at(const lbm_ctx *c, int64_t t) {
  const bool even = t % 2 == 0;
  switch (c->pattern) {
    case LBM_STREAM_PUSH: return G_NATURAL;
    case LBM_STREAM_AA: return even ? G_NATURAL : G_AA_ODD;
    case LBM_STREAM_ESOTERIC_PULL: return even ? G_ESO_EVEN : G_ESO_ODD;
    case LBM_STREAM_ESOTERIC_TWIST: return even ? G_TW_EVEN : G_TW_ODD;
  }
  return G_SHIFTED;
}

// one step with the context's current state; advances cur / t
static lbm_status one_step(lbm_ctx *c, int sp_override = -1) {
  const int sp = sp_override >= 0 ? sp_override : c->space;
  const int reg = sp_override >= 0 ? 0 : (c->reg ? 1 : 0);
  const int eq = sp_override >= 0 ? MAXWELL : c->eq;
  const int pat = step_pattern(c, c->t);
  const void *src;
  void *dst;
  if (two_buffers(c)) {
    src = c->buf[c->cur];
    dst = c->buf[c->cur ^ 1];
  } else {
    src = c->buf[0];
    dst = c->buf[0];
  }
  if (forced(c) && sp_override < 0) {
    // with a force the first-order deviations are -F/2, so the blocks from order 1 act too
    const bool cross = c->R.cross || c->R.cross1;
    const void *fn = cross ? sweep_force_cross_fn(c->s, c->store, pat) : sweep_force_fn(c->s, c->store, sp, pat);
    if (!fn) return fail(LBM_EUNSUPPORTED, "no forced kernel for this method");
    HIPCHECK(launch_sweep(c, fn, src, dst, false), "sweep launch");
  } else if (c->literal && sp_override < 0) {
    const void *fn = c->R.cross ? sweep_literal_cross_fn(c->s, c->store, c->form) : sweep_literal_fn(c->s, c->store, sp, c->form);
    if (!fn) return fail(LBM_EUNSUPPORTED, "no literal-arithmetic kernel for this method");
    HIPCHECK(launch_sweep(c, fn, src, dst, false), "sweep launch");
  } else if (c->transform == LBM_TRANSFORM_DENSE_MFMA && sp_override < 0) {
    const void *fn = sweep_mfma_fn(c->s, c->store, sp, reg);
    if (!fn) return fail(LBM_EUNSUPPORTED, "no MFMA ablation kernel for this method");
    HIPCHECK(launch_sweep_lds(c, fn, src, dst, mfma_lds_bytes(c)), "sweep launch");
  } else if (c->R.cross && sp_override < 0) {
    // an orthogonal raw basis: the general raw kernel with the cross-order blocks
    const void *fn = sweep_cross_fn(c->s, c->store, pat);
    if (!fn) return fail(LBM_EUNSUPPORTED, "no cross-order kernel for this stencil");
    HIPCHECK(launch_sweep(c, fn, src, dst, false), "sweep launch");
  } else if (c->stage && pat == PULL && stage_ok(c, c->bx, c->by)) {
    const void *fn = sweepl_fn(c->s, c->store, sp, eq, reg, c->bx);
    if (!fn) return fail(LBM_EUNSUPPORTED, "no LDS-staged sweep kernel for this method");
    const int lds = std::max(c->lds, sweepl_lds_bytes(c->s, c->store, c->bx));
    HIPCHECK(launch_sweep_lds(c, fn, src, dst, lds), "sweep launch");
  } else if (c->stage && pat == AA_ODD && stage_ok(c, c->bx, c->by)) {
    const void *fn = sweep_aa_shift_fn(c->s, c->store, sp, eq, reg);
    if (!fn) return fail(LBM_EUNSUPPORTED, "no LDS-shifted AA kernel for this method");
    const int lds = std::max(c->lds, aa_shift_lds_bytes(c, c->bx, c->by));
    HIPCHECK(launch_sweep_lds(c, fn, src, dst, lds), "sweep launch");
  } else {
    const bool vec = c->vec && (pat == PULL || pat == AA_EVEN) && vec_ok(c, c->bx);
    const void *fn = vec ? sweepv_fn(c->s, c->store, sp, eq, reg, pat) : sweep_fn(c->s, c->store, sp, eq, reg, pat);
    if (!fn) return fail(LBM_EUNSUPPORTED, "no sweep kernel for this method");
    HIPCHECK(launch_sweep(c, fn, src, dst, vec), "sweep launch");
  }
  if (two_buffers(c)) c->cur ^= 1;
  c->t += 1;
  return LBM_OK;
}

static int state_gather_mode(const lbm_ctx *c) { return gather_mode_at(c, c->t); }
static void *state_buffer(const lbm_ctx *c) { return two_buffers(c) ? c->buf[c->cur] : c->buf[0]; }

static FieldArgs field_args(const lbm_ctx *c, void *buf, int fbx, int fby) {
  FieldArgs a;
  std::memset(&a, 0, sizeof(a));
  a.buf = buf;
  a.L = c->L;
  a.absolute = c->p.zero_centered ? 0 : 1;
  a.forced = forced(c) ? 1 : 0;
  a.ffield = c->ffield;
  a.ffield_f64 = c->store == F64 ? 1 : 0;
  for (int d = 0; d < 3; ++d) a.fconst[d] = c->p.force[d];
  a.ncells = c->ncells;
  a.nx = c->nx;
  a.ny = c->ny;
  a.nz = c->nz;
  a.tiles_x = (c->nx + fbx - 1) / fbx;
  a.tiles_y = (c->ny + fby - 1) / fby;
  a.grav = c->p.gravity;
  return a;
}

static const int FBX = 64, FBY = 4;
static dim3 field_grid(const FieldArgs &a, int nz) { return dim3(unsigned(uint64_t(a.tiles_x) * a.tiles_y * nz)); }

static lbm_status launch_field(lbm_ctx *c, const void *fn, FieldArgs &a) {
  if (!fn) return fail(LBM_EUNSUPPORTED, "no kernel for this layout");
  void *args[] = {&a};
  HIPCHECK(hipLaunchKernel(fn, field_grid(a, c->nz), dim3(FBX, FBY), args, 0, c->stream), "field kernel launch");
  return LBM_OK;
}

static lbm_status ensure_staging(lbm_ctx *c, size_t ndoubles) {
  if (c->staging_doubles >= ndoubles) return LBM_OK;
  if (c->staging) {
    HIPCHECK(hipStreamSynchronize(c->stream), "sync");
    (void)hipFree(c->staging);
    c->staging = nullptr;
    c->staging_doubles = 0;
  }
  hipError_t e = hipMalloc(&c->staging, ndoubles * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(LBM_ENOMEM, "staging allocation failed");
  }
  c->staging_doubles = ndoubles;
  return LBM_OK;
}

static void clear_graphs(lbm_ctx *c) {
  for (auto &kv : c->gcache) (void)hipGraphExecDestroy(kv.second);
  c->gcache.clear();
}

static lbm_status check_ctx(const lbm_ctx *c) {
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  return LBM_OK;
}

}  // namespace lbm

// =======================================================================================
// C ABI
// =======================================================================================
extern "C" lbm_status lbm_create(const lbm_params *p, lbm_ctx **out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status s = validate(p);
  if (s != LBM_OK) return s;
  lbm_ctx *c = new lbm_ctx();
  c->p = *p;
  c->omegas.assign(p->omegas, p->omegas + p->n_omegas);
  c->p.omegas = c->omegas.data();
  c->s = p->stencil;
  c->q = stencil_q(p->stencil);
  c->d = stencil_d(p->stencil);
  c->space = internal_space(p->space);
  c->literal = p->arithmetic == LBM_ARITH_LITERAL;
  c->form = literal_form(p);
  c->eq = p->equilibrium == LBM_EQ_SHALLOW_WATER ? SWE
          : (p->equilibrium == LBM_EQ_SHALLOW_WATER_CONTINUOUS ? SWEK : MAXWELL);
  c->store = p->storage;
  c->pattern = p->streaming;
  c->nx = int(p->nx);
  c->ny = int(p->ny);
  c->nz = int(p->nz);
  c->ncells = uint32_t(p->nx * p->ny * p->nz);
  c->elem = storage_bytes(p->storage);
  s = relaxation_blocks(c->s, p->basis, c->omegas.data(), &c->R);
  if (s != LBM_OK) {
    delete c;
    return s;
  }
  c->reg = c->R.regularized;
  c->nbuf = two_buffers(c) ? 2 : 1;
  {
    uint64_t ps, zs, ys, elems;
    storage_strides(p, &ps, &zs, &ys, &elems);
    c->L.ps = ps;
    c->L.zs = zs;
    c->L.ys = uint32_t(ys);
    c->layout = resolve_layout(p);
    c->buf_bytes = size_t(elems) * c->elem;
  }
  {
    size_t need = 0;
    for (int k = 0; k < c->nbuf; ++k)
      if (!p->buffers[k]) need += c->buf_bytes;
    if (need) {
      s = check_free_memory(need, "population buffer");
      if (s != LBM_OK) {
        delete c;
        return s;
      }
    }
  }
  for (int k = 0; k < c->nbuf; ++k) {
    if (p->buffers[k]) {
      if (!is_device_ptr(p->buffers[k])) {
        delete c;
        return fail(LBM_EINVAL, "caller buffer " + std::to_string(k) + " is not device memory");
      }
      if (p->buffer_bytes < c->buf_bytes) {
        delete c;
        return fail(LBM_ENOMEM, "caller buffer smaller than q * ncells * sizeof(storage)");
      }
      c->buf[k] = p->buffers[k];
      c->own[k] = false;
    } else {
      hipError_t e = hipMalloc(&c->buf[k], c->buf_bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        lbm_destroy(c);
        return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,
                    std::string("population buffer allocation: ") + hipGetErrorString(e));
      }
      c->own[k] = true;
    }
  }
  if (p->stream) {
    c->stream = static_cast<hipStream_t>(p->stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      lbm_destroy(c);
      return hip_fail(e, "stream creation");
    }
    c->own_stream = true;
  }
  // default launch shape: 256 threads, as wide along x as the row allows
  int bx = 64;
  while (bx < 256 && bx < c->nx) bx *= 2;
  c->bx = bx;
  c->by = std::max(1, 256 / bx);
  c->swz = 0;
  c->diag_blocks = int(std::min<uint64_t>(2048, (uint64_t(c->ncells) + DIAG_THREADS - 1) / DIAG_THREADS));
  if (hipError_t ed = hipGetDevice(&c->device); ed != hipSuccess) {
    lbm_destroy(c);
    return hip_fail(ed, "current device");
  }
  hipError_t e = hipMalloc(&c->partials, (size_t(c->diag_blocks) * 6 + 8) * sizeof(double));
  if (e != hipSuccess) {
    lbm_destroy(c);
    return hip_fail(e, "partials allocation");
  }
  *out = c;
  return LBM_OK;
}

extern "C" void lbm_destroy(lbm_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  clear_graphs(c);
  for (int k = 0; k < 2; ++k)
    if (c->own[k] && c->buf[k]) (void)hipFree(c->buf[k]);
  if (c->staging) (void)hipFree(c->staging);
  if (c->partials) (void)hipFree(c->partials);
  if (c->ffield) (void)hipFree(c->ffield);
  free_tiles(c);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

extern "C" lbm_status lbm_init_equilibrium(lbm_ctx *c, const double *rho, const double *u) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (!rho || !u) return fail(LBM_EINVAL, "rho and u must be non-NULL");
  const size_t n = c->ncells;
  const double *drho = rho, *du = u;
  bool host = !is_device_ptr(rho) || !is_device_ptr(u);
  if (host) {
    lbm_status s = ensure_staging(c, 4 * n);
    if (s != LBM_OK) return s;
    HIPCHECK(hipMemcpyAsync(c->staging, rho, n * sizeof(double), hipMemcpyDefault, c->stream), "copy rho");
    HIPCHECK(hipMemcpyAsync(c->staging + n, u, size_t(c->d) * n * sizeof(double), hipMemcpyDefault, c->stream),
             "copy u");
    if (c->d == 2) HIPCHECK(hipMemsetAsync(c->staging + 3 * n, 0, n * sizeof(double), c->stream), "zero u_z");
    drho = c->staging;
    du = c->staging + n;
  }
  c->t = 0;
  c->cur = 0;
  const int gm = gather_mode_at(c, 0);
  const int sp_init = c->eq == SWE ? CENTRAL : c->space;
  FieldArgs a = field_args(c, c->buf[0], FBX, FBY);
  a.rho_in = drho;
  a.u_in = du;
  lbm_status s = launch_field(c, init_fn(c->s, c->store, sp_init, c->eq, gm), a);
  if (s != LBM_OK) return s;
  if (host) HIPCHECK(hipStreamSynchronize(c->stream), "init sync");
  return LBM_OK;
}

namespace lbm {
// Time loops are recorded in chunks of at most GRAPH_CHUNK steps (even, so a chunk keeps the
// buffer parity); lbm_step(n) replays the chunk graph n / GRAPH_CHUNK times and a graph of the
// remainder.  At most GRAPH_CACHE_MAX graphs are kept per context or batch; recording one more
// drops them all.
static const int64_t GRAPH_CHUNK = 256;
static const size_t GRAPH_CACHE_MAX = 8;

// the cached hipGraph that replays n sweeps from the current buffer parity (recorded once)
static lbm_status graph_for(lbm_ctx *c, int64_t n, hipGraphExec_t *out) {
  const int parity = two_buffers(c) ? c->cur : int(c->t % 2);
  auto key = std::make_pair(n, parity);
  auto it = c->gcache.find(key);
  if (it == c->gcache.end()) {
    if (c->gcache.size() >= GRAPH_CACHE_MAX) {
      HIPCHECK(hipStreamSynchronize(c->stream), "sync before graph eviction");
      clear_graphs(c);
    }
    const int cur0 = c->cur;
    const int64_t t0 = c->t;
    lbm_status st = ensure_tiles(c);
    if (st != LBM_OK) return st;
    HIPCHECK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    lbm_status s = LBM_OK;
    for (int64_t k = 0; k < n && s == LBM_OK; ++k) s = one_step(c);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->cur = cur0;
    c->t = t0;
    if (s != LBM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    it = c->gcache.emplace(key, ex).first;
  }
  *out = it->second;
  return LBM_OK;
}
}  // namespace lbm

extern "C" lbm_status lbm_step(lbm_ctx *c, int64_t n) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  if (n == 0) return LBM_OK;
  if (!c->graphs || n < 2) {
    lbm_status st = ensure_tiles(c);
    if (st != LBM_OK) return st;
    for (int64_t k = 0; k < n; ++k) {
      lbm_status s = one_step(c);
      if (s != LBM_OK) return s;
    }
    return LBM_OK;
  }
  while (n >= 2) {
    const int64_t m = std::min(n, GRAPH_CHUNK);
    hipGraphExec_t ex = nullptr;
    lbm_status s = graph_for(c, m, &ex);
    if (s != LBM_OK) return s;
    HIPCHECK(hipGraphLaunch(ex, c->stream), "graph launch");
    if (two_buffers(c)) c->cur ^= int(m & 1);
    c->t += m;
    n -= m;
  }
  if (n == 1) {
    lbm_status st = ensure_tiles(c);
    if (st == LBM_OK) st = one_step(c);
    return st;
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_graph_prepare(lbm_ctx *c, int64_t n) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (n < 2 || !c->graphs) return LBM_OK;
  // the chunk graph and the remainder graph (chunks are even: same parity)
  hipGraphExec_t ex = nullptr;
  lbm_status s = graph_for(c, std::min(n, GRAPH_CHUNK), &ex);
  if (s == LBM_OK && n > GRAPH_CHUNK && n % GRAPH_CHUNK >= 2) s = graph_for(c, n % GRAPH_CHUNK, &ex);
  return s;
}

extern "C" lbm_status lbm_debug_stream_only(lbm_ctx *c, int64_t n) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  lbm_status st = ensure_tiles(c);
  if (st != LBM_OK) return st;
  for (int64_t k = 0; k < n; ++k) {
    lbm_status s = one_step(c, IDENTITY);
    if (s != LBM_OK) return s;
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_set_force_field(lbm_ctx *c, const double *F) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  HIPCHECK(hipStreamSynchronize(c->stream), "force sync");
  clear_graphs(c);
  if (!F) {
    if (c->ffield) (void)hipFree(c->ffield);
    c->ffield = nullptr;
    return LBM_OK;
  }
  if (c->eq != MAXWELL) return fail(LBM_EUNSUPPORTED, "the body force is implemented with the Maxwellian equilibrium");
  if (c->literal) return fail(LBM_EUNSUPPORTED, "the body force runs with the deviation arithmetic");
  if (c->transform == LBM_TRANSFORM_DENSE_MFMA) return fail(LBM_EUNSUPPORTED, "no body force in the MFMA ablation");
  const size_t n = 3 * size_t(c->ncells);
  std::vector<double> h(n);
  if (is_device_ptr(F)) HIPCHECK(hipMemcpy(h.data(), F, n * sizeof(double), hipMemcpyDeviceToHost), "force copy");
  else std::memcpy(h.data(), F, n * sizeof(double));
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(h[k])) return fail(LBM_EINVAL, "the force field must be finite");
  const size_t eb = c->store == F64 ? sizeof(double) : sizeof(float);
  if (!c->ffield) {
    hipError_t e = hipMalloc(&c->ffield, n * eb);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      c->ffield = nullptr;
      return fail(LBM_ENOMEM, "force field allocation");
    }
  }
  if (c->store == F64) {
    HIPCHECK(hipMemcpy(c->ffield, h.data(), n * sizeof(double), hipMemcpyHostToDevice), "force upload");
  } else {
    std::vector<float> hf(n);
    for (size_t k = 0; k < n; ++k) hf[k] = float(h[k]);
    HIPCHECK(hipMemcpy(c->ffield, hf.data(), n * sizeof(float), hipMemcpyHostToDevice), "force upload");
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_macroscopic(lbm_ctx *c, double *rho, double *u) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (!rho || !u) return fail(LBM_EINVAL, "rho and u must be non-NULL");
  const size_t n = c->ncells;
  const bool dev = is_device_ptr(rho) && is_device_ptr(u);
  double *r = rho, *v = u;
  if (!dev) {
    lbm_status s = ensure_staging(c, 4 * n);
    if (s != LBM_OK) return s;
    r = c->staging;
    v = c->staging + n;
  }
  FieldArgs a = field_args(c, state_buffer(c), FBX, FBY);
  a.rho_out = r;
  a.u_out = v;
  lbm_status s = launch_field(c, macro_fn(c->s, c->store, state_gather_mode(c)), a);
  if (s != LBM_OK) return s;
  if (!dev) {
    HIPCHECK(hipMemcpyAsync(rho, r, n * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy rho");
    // all three components: the kernel writes u_z = 0 for D2Q9
    HIPCHECK(hipMemcpyAsync(u, v, 3 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy u");
  }
  HIPCHECK(hipStreamSynchronize(c->stream), "macroscopic sync");
  return LBM_OK;
}

static lbm_status transfer_populations(lbm_ctx *c, double *df, bool to_host_layout) {
  const size_t n = c->ncells;
  const bool dev = is_device_ptr(df);
  const int gm = state_gather_mode(c);
  const void *fn = to_host_layout ? export_fn(c->s, c->store, gm) : import_fn(c->s, c->store, gm);
  if (dev) {
    FieldArgs a = field_args(c, state_buffer(c), FBX, FBY);
    a.pop = df;
    a.i0 = 0;
    a.i1 = c->q;
    lbm_status s = launch_field(c, fn, a);
    if (s != LBM_OK) return s;
    HIPCHECK(hipStreamSynchronize(c->stream), "population sync");
    return LBM_OK;
  }
  const size_t budget = size_t(256) << 20;  // bytes of staging per chunk
  int per = int(std::max<size_t>(1, budget / (n * sizeof(double))));
  per = std::min(per, c->q);
  lbm_status s = ensure_staging(c, size_t(per) * n);
  if (s != LBM_OK) return s;
  for (int i0 = 0; i0 < c->q; i0 += per) {
    const int i1 = std::min(c->q, i0 + per);
    const size_t bytes = size_t(i1 - i0) * n * sizeof(double);
    if (!to_host_layout)
      HIPCHECK(hipMemcpyAsync(c->staging, df + size_t(i0) * n, bytes, hipMemcpyHostToDevice, c->stream), "copy in");
    FieldArgs a = field_args(c, state_buffer(c), FBX, FBY);
    a.pop = c->staging;
    a.i0 = i0;
    a.i1 = i1;
    s = launch_field(c, fn, a);
    if (s != LBM_OK) return s;
    if (to_host_layout)
      HIPCHECK(hipMemcpyAsync(df + size_t(i0) * n, c->staging, bytes, hipMemcpyDeviceToHost, c->stream), "copy out");
    HIPCHECK(hipStreamSynchronize(c->stream), "population sync");
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_get_populations(lbm_ctx *c, double *df) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (!df) return fail(LBM_EINVAL, "df is NULL");
  return transfer_populations(c, df, true);
}

extern "C" lbm_status lbm_set_populations(lbm_ctx *c, const double *df) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (!df) return fail(LBM_EINVAL, "df is NULL");
  return transfer_populations(c, const_cast<double *>(df), false);
}

extern "C" lbm_status lbm_diagnostics(lbm_ctx *c, double out[6]) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  FieldArgs a = field_args(c, state_buffer(c), FBX, FBY);
  a.partials = c->partials;
  const void *fn = diag_fn(c->s, c->store, state_gather_mode(c));
  if (!fn) return fail(LBM_EUNSUPPORTED, "no diagnostics kernel");
  void *args[] = {&a};
  HIPCHECK(hipLaunchKernel(fn, dim3(c->diag_blocks), dim3(DIAG_THREADS), args, 0, c->stream), "diag launch");
  double *dout = c->partials + size_t(c->diag_blocks) * 6;
  int nb = c->diag_blocks;
  void *args2[] = {&c->partials, &nb, &dout};
  HIPCHECK(hipLaunchKernel(diag_final_fn(), dim3(1), dim3(DIAG_THREADS), args2, 0, c->stream), "diag final launch");
  HIPCHECK(hipMemcpyAsync(out, dout, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "diag copy");
  HIPCHECK(hipStreamSynchronize(c->stream), "diag sync");
  if (out[5] > 0.0) return fail(LBM_ENONFINITE, "non-finite populations found");
  return LBM_OK;
}

// ---------------------------------------------------------------------------------------
// allocation-free diagnostics: the partial sums live in a static device array (one copy per
// GPU, kept until the process ends) instead of the context's buffer
// ---------------------------------------------------------------------------------------
namespace lbm {
static constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(LBM_NOALLOC_SCRATCH_BYTES) / sizeof(double);
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
static constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[MAX_DEVICES] = {};

// Device address of this GPU's scratch array; looked up once per device, with that device
// current (the host-side name of the array is not a device address).
static lbm_status scratch_ptr(int device, double **out) {
  if (device < 0 || device >= MAX_DEVICES) return fail(LBM_EDEVICE, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "scratch symbol address");
    g_scratch_dev[device] = static_cast<double *>(p);
  }
  *out = g_scratch_dev[device];
  return LBM_OK;
}
}  // namespace lbm

extern "C" lbm_status lbm_diagnostics_noalloc(lbm_ctx *c, double *out) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev), "current device");
  if (dev != c->device) return fail(LBM_EINVAL, "the context's device must be current");
  const int nb = c->diag_blocks;
  const size_t need = size_t(nb) * 6 + 6;  // partials, then the six sums for a host destination
  if (need > NOALLOC_SCRATCH_DOUBLES)
    return fail(LBM_EUNSUPPORTED, "the reduction needs " + std::to_string(need * sizeof(double)) +
                                      " bytes of scratch, more than the " +
                                      std::to_string(LBM_NOALLOC_SCRATCH_BYTES) + " the library holds");
  double *sp = nullptr;
  lbm_status st = scratch_ptr(dev, &sp);
  if (st != LBM_OK) return st;
  const void *fn = diag_fn(c->s, c->store, state_gather_mode(c));
  if (!fn) return fail(LBM_EUNSUPPORTED, "no diagnostics kernel");
  // every block writes all six of its partials and the final kernel reads exactly nb blocks,
  // so nothing left in the array by an earlier call is read
  FieldArgs a = field_args(c, state_buffer(c), FBX, FBY);
  a.partials = sp;
  void *args[] = {&a};
  HIPCHECK(hipLaunchKernel(fn, dim3(nb), dim3(DIAG_THREADS), args, 0, c->stream), "diag launch");
  const bool dev_out = is_device_ptr(out);
  double *dout = dev_out ? out : sp + size_t(nb) * 6;
  int nbv = nb;
  void *args2[] = {&sp, &nbv, &dout};
  HIPCHECK(hipLaunchKernel(diag_final_fn(), dim3(1), dim3(DIAG_THREADS), args2, 0, c->stream), "diag final launch");
  if (dev_out) return LBM_OK;
  HIPCHECK(hipMemcpyAsync(out, dout, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "diag copy");
  HIPCHECK(hipStreamSynchronize(c->stream), "diag sync");
  if (out[5] > 0.0) return fail(LBM_ENONFINITE, "non-finite populations found");
  return LBM_OK;
}

extern "C" lbm_status lbm_synchronize(lbm_ctx *c) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  HIPCHECK(hipStreamSynchronize(c->stream), "synchronize");
  return LBM_OK;
}

extern "C" int64_t lbm_time(const lbm_ctx *c) { return c ? c->t : -1; }

extern "C" lbm_status lbm_set_time(lbm_ctx *c, int64_t t) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (t < 0) return fail(LBM_EINVAL, "t must be >= 0");
  if (!two_buffers(c) && (t % 2) != (c->t % 2)) {
    // odd and even times use different layouts: move the state pair by pair (slots i and
    // opp(i) only exchange with each other) from the old layout to the new one
    const size_t n = c->ncells;
    lbm_status s = ensure_staging(c, 2 * n);
    if (s != LBM_OK) return s;
    const int gm_old = state_gather_mode(c);
    const int gm_new = gather_mode_at(c, t);
    for (int i0 = 0; i0 < c->q; i0 = (i0 == 0 ? 1 : i0 + 2)) {
      FieldArgs a = field_args(c, c->buf[0], FBX, FBY);
      a.pop = c->staging;
      a.i0 = i0;
      a.i1 = i0 == 0 ? 1 : i0 + 2;
      s = launch_field(c, export_fn(c->s, c->store, gm_old), a);
      if (s == LBM_OK) s = launch_field(c, import_fn(c->s, c->store, gm_new), a);
      if (s != LBM_OK) return s;
    }
    HIPCHECK(hipStreamSynchronize(c->stream), "relayout sync");
  }
  clear_graphs(c);
  c->t = t;
  return LBM_OK;
}

extern "C" lbm_status lbm_set_launch(lbm_ctx *c, int bx, int by, int swz) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (bx < 1 || by < 1 || (bx * by) % 64 != 0 || bx * by > 512)
    return fail(LBM_EINVAL, "bx * by must be a positive multiple of 64 and at most 512");
  if (c->bx != bx || c->by != by || c->swz != (swz ? 1 : 0)) clear_graphs(c);
  c->bx = bx;
  c->by = by;
  c->swz = swz ? 1 : 0;
  if (c->vec && !vec_ok(c, bx)) c->vec = false;
  if (c->stage && !stage_ok(c, bx, by)) c->stage = false;
  if (c->transform == LBM_TRANSFORM_DENSE_MFMA && bx * by > 256) c->transform = LBM_TRANSFORM_CHIMERA;
  return LBM_OK;
}

extern "C" lbm_status lbm_set_vectorized(lbm_ctx *c, int enable) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (enable && !vec_ok(c, c->bx))
    return fail(LBM_EUNSUPPORTED, "the vectorised sweep needs nx to be a multiple of bx * V (V = 2 for F64/F32, 4 for F16)");
  if (c->vec != (enable != 0)) clear_graphs(c);
  c->vec = enable != 0;
  return LBM_OK;
}

extern "C" int lbm_get_vectorized(const lbm_ctx *c) { return c && c->vec ? 1 : 0; }

extern "C" lbm_status lbm_set_staged(lbm_ctx *c, int enable) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (enable && !stage_ok(c, c->bx, c->by))
    return fail(LBM_EUNSUPPORTED, "the LDS variant needs the pull pattern with blocks of 128 x 1 or 256 x 1 "
                                  "threads, nx a multiple of bx and 16-byte aligned buffers, or the AA pattern "
                                  "with at most 256 threads and nx a multiple of bx");
  if (c->stage != (enable != 0)) clear_graphs(c);
  c->stage = enable != 0;
  return LBM_OK;
}

extern "C" int lbm_get_staged(const lbm_ctx *c) { return c && c->stage ? 1 : 0; }

extern "C" lbm_status lbm_set_transform(lbm_ctx *c, int transform) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (transform != LBM_TRANSFORM_CHIMERA && transform != LBM_TRANSFORM_DENSE_MFMA)
    return fail(LBM_EINVAL, "transform out of range");
  if (transform == LBM_TRANSFORM_DENSE_MFMA) {
    if (c->s != LBM_D3Q27 || c->pattern != LBM_STREAM_PULL || c->eq != MAXWELL || c->space == SRT || c->literal ||
        forced(c) || c->R.cross)
      return fail(LBM_EUNSUPPORTED,
                  "the MFMA ablation covers D3Q27 moment spaces, pull streaming, Maxwellian equilibrium, "
                  "deviation arithmetic, the graded basis");
    if (c->bx * c->by > 256 || (c->bx * c->by) % 64 != 0)
      return fail(LBM_EUNSUPPORTED, "the MFMA ablation needs blocks of 64..256 threads (whole waves)");
  }
  if (c->transform != transform) clear_graphs(c);
  c->transform = transform;
  return LBM_OK;
}

extern "C" int lbm_get_transform(const lbm_ctx *c) { return c ? c->transform : -1; }

extern "C" int lbm_get_layout(const lbm_ctx *c) { return c ? c->layout : -1; }

extern "C" lbm_status lbm_set_lds_reserve(lbm_ctx *c, int bytes) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (bytes < 0 || bytes > 65536) return fail(LBM_EINVAL, "LDS reserve must be in [0, 65536] bytes");
  if (c->lds != bytes) clear_graphs(c);
  c->lds = bytes;
  return LBM_OK;
}

extern "C" int lbm_get_lds_reserve(const lbm_ctx *c) { return c ? c->lds : -1; }

extern "C" lbm_status lbm_get_launch(const lbm_ctx *c, int *bx, int *by, int *swz) {
  if (!c || !bx || !by || !swz) return fail(LBM_EINVAL, "NULL argument");
  *bx = c->bx;
  *by = c->by;
  *swz = c->swz;
  return LBM_OK;
}

extern "C" lbm_status lbm_set_graphs(lbm_ctx *c, int enable) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  c->graphs = enable != 0;
  return LBM_OK;
}

extern "C" lbm_status lbm_buffer(const lbm_ctx *c, int k, void **ptr, size_t *bytes) {
  if (!c || !ptr) return fail(LBM_EINVAL, "NULL argument");
  if (k < 0 || k >= c->nbuf) return fail(LBM_EINVAL, "buffer index out of range");
  *ptr = c->buf[k];
  if (bytes) *bytes = c->buf_bytes;
  return LBM_OK;
}

extern "C" lbm_status lbm_time_steps(lbm_ctx *c, int64_t n, double *ms) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  if (!ms) return fail(LBM_EINVAL, "ms is NULL");
  EventPair ev;
  HIPCHECK(ev.create(), "event");
  HIPCHECK(hipEventRecord(ev.e0, c->stream), "event record");
  lbm_status s = lbm_step(c, n);
  HIPCHECK(hipEventRecord(ev.e1, c->stream), "event record");
  float f = 0.f;
  HIPCHECK(ev.elapsed(&f), "elapsed");
  *ms = double(f);
  return s;
}

// ---------------------------------------------------------------------------------------
// autotuning of the launch shape
// ---------------------------------------------------------------------------------------
static std::string tune_key(const lbm_ctx *c) {
  std::ostringstream k;
  k << "s" << c->s << "_sp" << c->space << "_eq" << c->eq << "_r" << int(c->reg) << "_st" << c->store << "_pat"
    << c->pattern << "_lay" << c->layout << (c->literal ? "_lit" + std::to_string(c->form) : std::string())
    << (c->p.zero_centered ? "" : "_abs") << (c->R.cross ? "_cross" : "") << (forced(c) ? "_force" : "")
    << (c->transform == LBM_TRANSFORM_DENSE_MFMA ? "_mfma" : "") << "_"
    << c->nx << "x" << c->ny << "x" << c->nz;
  return k.str();
}

static bool cache_lookup(const std::string &file, const std::string &key, int *bx, int *by, int *swz, int *vec,
                         int *lds) {
  std::ifstream in(file);
  if (!in) return false;
  std::string line;
  const std::string pat = "\"" + key + "\"";
  while (std::getline(in, line)) {
    size_t p = line.find(pat);
    if (p == std::string::npos) continue;
    size_t lb = line.find('[', p);
    if (lb == std::string::npos) continue;
    double ms = 0;
    if (std::sscanf(line.c_str() + lb, "[%d, %d, %d, %d, %d, %lf", bx, by, swz, vec, lds, &ms) >= 5) return true;
  }
  return false;
}

static void cache_store(const std::string &file, const std::string &key, int bx, int by, int swz, int vec, int lds,
                        double ms) {
  // keep every other "key": [values] pair of the file, whatever its line layout
  std::vector<std::pair<std::string, std::string>> kept;
  {
    std::ifstream in(file);
    std::ostringstream ss;
    ss << in.rdbuf();
    const std::string text = ss.str();
    size_t p = 0;
    for (;;) {
      const size_t k0 = text.find('"', p);
      if (k0 == std::string::npos) break;
      const size_t k1 = text.find('"', k0 + 1);
      if (k1 == std::string::npos) break;
      const size_t lb = text.find('[', k1);
      const size_t rb = lb == std::string::npos ? std::string::npos : text.find(']', lb);
      if (rb == std::string::npos) break;
      std::string k = text.substr(k0 + 1, k1 - k0 - 1);
      if (k != key) kept.emplace_back(std::move(k), text.substr(lb, rb - lb + 1));
      p = rb + 1;
    }
  }
  char buf[128];
  std::snprintf(buf, sizeof(buf), "[%d, %d, %d, %d, %d, %.6f]", bx, by, swz, vec, lds, ms);
  kept.emplace_back(key, buf);
  std::ofstream out(file, std::ios::trunc);
  out << "{\n";
  for (size_t i = 0; i < kept.size(); ++i)
    out << "  \"" << kept[i].first << "\": " << kept[i].second << (i + 1 < kept.size() ? ",\n" : "\n");
  out << "}\n";
}

extern "C" lbm_status lbm_autotune(lbm_ctx *c) {
  if (check_ctx(c) != LBM_OK) return LBM_EINVAL;
  const char *file = std::getenv("LBM_AUTOTUNE_CACHE");
  const std::string key = tune_key(c);
  // the MFMA ablation kernel takes blocks of at most four waves, stages its own tiles in LDS
  // and has no vectorised form
  const bool mfma = c->transform == LBM_TRANSFORM_DENSE_MFMA;
  const int max_threads = mfma ? 256 : 512;
  int bx, by, swz, vec = 0, lds = 0;
  // kernel variant of a shape: 0 per-cell registers, 1 vectorised, 2 LDS-staged (pull)
  auto apply_variant = [&](int v) {
    lbm_status r = lbm_set_vectorized(c, v == 1 ? 1 : 0);
    return r != LBM_OK ? r : lbm_set_staged(c, v == 2 ? 1 : 0);
  };
  if (file && cache_lookup(file, key, &bx, &by, &swz, &vec, &lds) && bx * by <= max_threads) {
    lbm_status s0 = lbm_set_launch(c, bx, by, swz);
    if (s0 == LBM_OK) s0 = apply_variant(mfma ? 0 : vec);
    if (s0 == LBM_OK) s0 = lbm_set_lds_reserve(c, mfma ? 0 : lds);
    if (s0 == LBM_OK) return LBM_OK;
    // the cached choice does not apply to this context (e.g. caller buffers without the
    // alignment the LDS variant needs): tune it afresh
    g_last_error.clear();
  }
  // candidate shapes: (bx, by, swizzle, variant)
  const bool plain = !mfma && !forced(c) && !c->literal && !c->R.cross;  // the default branch of one_step
  std::vector<std::array<int, 4>> cand;
  for (int cbx : {64, 128, 256, 512})
    for (int cby : {1, 2, 4, 8})
      for (int cs : {0, 1})
        for (int cv : {0, 1, 2}) {
          if (cbx * cby > max_threads || (cbx * cby) % 64 != 0) continue;
          if (cv == 1 && (mfma || cbx * cby > 256 || !vec_ok(c, cbx))) continue;
          if (cv == 2 && (!plain || !stage_ok(c, cbx, cby))) continue;
          if (cbx > 64 && cbx / 2 >= c->nx) continue;
          if (cby > 1 && cby / 2 >= c->ny) continue;
          cand.push_back({cbx, cby, cs, cv});
        }
  // the sweep must leave the state unchanged: pull and push write only the other buffer, so
  // every timed sweep repeats the same src -> dst step; the in-place patterns run on a copy of
  // the buffer that is restored afterwards and time their even and odd steps alternately, as
  // they run, over an even number of steps
  const bool two = two_buffers(c);
  EventPair ev;
  HIPCHECK(ev.create(), "event");
  void *saved = nullptr;
  if (!two) {
    hipError_t e = hipMalloc(&saved, c->buf_bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(saved, c->buf[0], c->buf_bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      if (saved) (void)hipFree(saved);
      return fail(LBM_ENOMEM, "autotuning the in-place pattern needs a temporary copy of the state");
    }
  }
  const int cur0 = c->cur;
  const int64_t t0 = c->t;
  const int bx0 = c->bx, by0 = c->by, swz0 = c->swz, lds0 = c->lds;
  const bool vec0 = c->vec, stage0 = c->stage;
  const bool g0 = c->graphs;
  c->lds = 0;
  c->graphs = false;
  const uint64_t lups = uint64_t(c->ncells);
  int reps = int(std::max<uint64_t>(4, std::min<uint64_t>(20, (uint64_t(1) << 27) / std::max<uint64_t>(1, lups) + 2)));
  reps += reps & 1;
  const bool verbose = std::getenv("LBM_AUTOTUNE_VERBOSE") != nullptr;
  // time `reps` sweeps (after one warm-up) of the shape cd with LDS reserve c->lds
  auto time_shape = [&](const std::array<int, 4> &cd, float *ms) -> lbm_status {
    c->bx = cd[0];
    c->by = cd[1];
    c->swz = cd[2];
    c->vec = cd[3] == 1;
    c->stage = cd[3] == 2;
    c->t = t0;
    lbm_status st = ensure_tiles(c);  // time the launch as lbm_step runs it, with its tile table
    for (int r = 0; r < reps + 1 && st == LBM_OK; ++r) {
      if (r == 1) (void)hipEventRecord(ev.e0, c->stream);
      c->cur = cur0;
      if (two) c->t = t0;
      st = one_step(c);
    }
    (void)hipEventRecord(ev.e1, c->stream);
    const hipError_t e = ev.elapsed(ms);
    if (st != LBM_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    if (verbose)
      std::fprintf(stderr, "[lbm autotune] %s bx %d by %d swizzle %d variant %d lds %d: %.4f ms/step\n", key.c_str(),
                   cd[0], cd[1], cd[2], cd[3], c->lds, *ms / reps);
    return LBM_OK;
  };
  double best = 1e300;
  int bb[4] = {bx0, by0, swz0, vec0 ? 1 : (stage0 ? 2 : 0)};
  int best_lds = 0;
  // best uncapped shape per block size (64, 128, 256, 512 threads), the starting points of phase 2
  double best_t[4] = {1e300, 1e300, 1e300, 1e300};
  std::array<int, 4> shape_t[4] = {};
  lbm_status st = LBM_OK;
  for (const auto &cd : cand) {
    float ms = 0.f;
    st = time_shape(cd, &ms);
    if (st != LBM_OK) break;
    if (ms < best) {
      best = ms;
      for (int k = 0; k < 4; ++k) bb[k] = cd[k];
    }
    const int ti = cd[0] * cd[1] == 64 ? 0 : cd[0] * cd[1] == 128 ? 1 : cd[0] * cd[1] == 256 ? 2 : 3;
    if (ms < best_t[ti]) {
      best_t[ti] = ms;
      shape_t[ti] = cd;
    }
  }
  // phase 2: occupancy cap (dynamic LDS per block) on the best shape of each block size.  Fewer
  // resident waves than the registers allow can stream faster, so the cap and the block size
  // are chosen together; the ladder holds at most 10, 8, 6, 5, 4, 3 or 2 blocks per CU (160 KiB).
  // The MFMA ablation sizes its LDS itself.
  for (int ti = 0; ti < 4 && st == LBM_OK && !mfma; ++ti) {
    if (best_t[ti] >= 1e300) continue;
    for (int l : {16384, 20480, 26624, 32768, 40960, 53248, 65536}) {
      c->lds = l;
      float ms = 0.f;
      st = time_shape(shape_t[ti], &ms);
      if (st != LBM_OK) break;
      if (ms < best) {
        best = ms;
        for (int k = 0; k < 4; ++k) bb[k] = shape_t[ti][k];
        best_lds = l;
      }
    }
  }
  // restore the state, the step counter and the previous launch on every path
  c->lds = lds0;
  c->cur = cur0;
  c->t = t0;
  c->graphs = g0;
  c->bx = bx0;
  c->by = by0;
  c->swz = swz0;
  c->vec = vec0;
  c->stage = stage0;
  if (saved) {
    const hipError_t e1 = hipMemcpyAsync(c->buf[0], saved, c->buf_bytes, hipMemcpyDeviceToDevice, c->stream);
    const hipError_t e2 = hipStreamSynchronize(c->stream);
    (void)hipFree(saved);
    if (st == LBM_OK && e1 != hipSuccess) return hip_fail(e1, "autotune state restore");
    if (st == LBM_OK && e2 != hipSuccess) return hip_fail(e2, "autotune state restore");
  }
  if (st != LBM_OK) return st;
  lbm_status s2 = lbm_set_launch(c, bb[0], bb[1], bb[2]);
  if (s2 == LBM_OK) s2 = apply_variant(bb[3]);
  if (s2 == LBM_OK) s2 = lbm_set_lds_reserve(c, best_lds);
  if (s2 == LBM_OK && file) cache_store(file, key, bb[0], bb[1], bb[2], bb[3], best_lds, best / reps);
  return s2;
}

extern "C" lbm_status lbm_copy_bandwidth(void *dst, const void *src, size_t bytes, int reps, void *stream, double *ms) {
  if (!dst || !src || !ms || reps < 1) return fail(LBM_EINVAL, "bad argument");
  if (bytes % 16 != 0) return fail(LBM_EINVAL, "bytes must be a multiple of 16");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t n = bytes / 16;
  if ((n + 255) / 256 > 0x7fffffffu) return fail(LBM_EINVAL, "copy too large for one launch");
  const unsigned blocks = unsigned((n + 255) / 256);
  EventPair ev;
  HIPCHECK(ev.create(), "event");
  lbm_v4u *d = static_cast<lbm_v4u *>(dst);
  const lbm_v4u *sp = static_cast<const lbm_v4u *>(src);
  void *args[] = {&d, &sp, const_cast<size_t *>(&n)};
  HIPCHECK(hipLaunchKernel(copy_fn(), dim3(blocks), dim3(256), args, 0, s), "copy launch");
  HIPCHECK(hipEventRecord(ev.e0, s), "event record");
  for (int r = 0; r < reps; ++r)
    HIPCHECK(hipLaunchKernel(copy_fn(), dim3(blocks), dim3(256), args, 0, s), "copy launch");
  HIPCHECK(hipEventRecord(ev.e1, s), "event record");
  float f = 0.f;
  HIPCHECK(ev.elapsed(&f), "elapsed");
  *ms = double(f);
  return LBM_OK;
}

// =======================================================================================
// batched ensemble
// =======================================================================================
#include "lbm_batch_kernels.hpp"

namespace lbm {
const void *batch_sweep_fn(int s, int store, int sp, int reg, bool persistent) {
  switch (s * 3 + store) {
    case 3: return BTable<D3Q19, F64>::sweep(sp, reg, persistent);
    case 4: return BTable<D3Q19, F32>::sweep(sp, reg, persistent);
    case 5: return BTable<D3Q19, F16>::sweep(sp, reg, persistent);
    case 6: return BTable<D3Q27, F64>::sweep(sp, reg, persistent);
    case 7: return BTable<D3Q27, F32>::sweep(sp, reg, persistent);
    case 8: return BTable<D3Q27, F16>::sweep(sp, reg, persistent);
  }
  return nullptr;
}
}  // namespace lbm

struct lbm_batch {
  lbm_params p;
  int s = 0, q = 0, d = 0, space = 0, store = 0;
  bool reg = true;
  size_t elem = 4;
  int nboxes = 0;
  std::vector<BoxInfo> boxes;
  uint32_t ntot = 0, ntiles = 0;
  uint64_t ntiles_cap = 0;  // capacity of tile_box_d
  BoxInfo *boxes_d = nullptr;
  uint32_t *tile_box_d = nullptr;
  void *relax_d = nullptr;
  void *buf[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t t = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool graphs = true;
  std::map<std::pair<int64_t, int>, hipGraphExec_t> gcache;
  double *staging = nullptr;
  size_t staging_doubles = 0;
  int swz = 1;  // XCD-ordered tiles (LBM_BATCH_SWIZZLE=0 switches it off)
  int bt = BATCH_THREADS;  // cells per tile = threads per block
  int lds = 0;             // dynamic LDS reserved per block (caps resident blocks per CU)
  bool persistent = false; // grid-stride loop over the tiles with a resident grid
  uint32_t pgrid = 0;      // its grid: resident blocks per CU x CUs, a multiple of 8
};

namespace lbm {

// Grid of the persistent form: the blocks that fit on the device at once for the current
// tile size and LDS reserve, rounded down to a multiple of 8 (one per XCD in turn).
static lbm_status batch_persistent_grid(lbm_batch *b) {
  const void *fn = batch_sweep_fn(b->s, b->store, b->space, b->reg ? 1 : 0, true);
  if (!fn) return fail(LBM_EUNSUPPORTED, "no batched sweep kernel for this method");
  int dev = 0, cus = 0, per_cu = 0;
  HIPCHECK(hipGetDevice(&dev), "current device");
  HIPCHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, b->bt, size_t(b->lds)), "occupancy");
  const uint32_t g = uint32_t(std::max(1, per_cu) * std::max(1, cus));
  b->pgrid = std::max<uint32_t>(8, g - g % 8);
  return LBM_OK;
}

static lbm_status batch_one_step(lbm_batch *b) {
  const void *fn = batch_sweep_fn(b->s, b->store, b->space, b->reg ? 1 : 0, b->persistent);
  if (!fn) return fail(LBM_EUNSUPPORTED, "no batched sweep kernel for this method");
  hipError_t e;
  auto go = [&](auto tag) {
    using ST = typename decltype(tag)::first_type;
    using CT = typename decltype(tag)::second_type;
    BatchArgs<ST, CT> a;
    a.src = static_cast<const ST *>(b->buf[b->cur]);
    a.dst = static_cast<ST *>(b->buf[b->cur ^ 1]);
    a.ntot = b->ntot;
    a.boxes = b->boxes_d;
    a.tile_box = b->tile_box_d;
    a.relax = static_cast<const Relax<CT> *>(b->relax_d);
    a.swizzle = b->swz;
    a.ntiles = b->ntiles;
    void *args[] = {&a};
    const unsigned grid = b->persistent ? std::min<unsigned>(b->pgrid, b->ntiles) : b->ntiles;
    return hipLaunchKernel(fn, dim3(grid), dim3(b->bt), args, size_t(b->lds), b->stream);
  };
  if (b->store == F64) e = go(std::pair<double, double>());
  else if (b->store == F32) e = go(std::pair<float, float>());
  else e = go(std::pair<_Float16, float>());
  HIPCHECK(e, "batched sweep launch");
  b->cur ^= 1;
  b->t += 1;
  return LBM_OK;
}

// tile table for tiles of bt cells: the first tile of every box and the box of every tile
static lbm_status batch_build_tiles(lbm_batch *b, int bt) {
  uint64_t tiles = 0;
  for (auto &B : b->boxes) {
    B.tile0 = uint32_t(tiles);
    tiles += (B.ncells + uint32_t(bt) - 1) / uint32_t(bt);
  }
  if (tiles >= (uint64_t(1) << 31)) return fail(LBM_EUNSUPPORTED, "too many tiles");
  std::vector<uint32_t> tb(tiles);
  for (size_t k = 0; k < b->boxes.size(); ++k) {
    const uint32_t nt = (b->boxes[k].ncells + uint32_t(bt) - 1) / uint32_t(bt);
    for (uint32_t j = 0; j < nt; ++j) tb[b->boxes[k].tile0 + j] = uint32_t(k);
  }
  if (b->stream) HIPCHECK(hipStreamSynchronize(b->stream), "sync");
  if (b->tile_box_d && tiles > b->ntiles_cap) {
    (void)hipFree(b->tile_box_d);
    b->tile_box_d = nullptr;
  }
  if (!b->tile_box_d) {
    hipError_t e = hipMalloc(&b->tile_box_d, sizeof(uint32_t) * tiles);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(LBM_ENOMEM, "tile table allocation failed");
    }
    b->ntiles_cap = tiles;
  }
  HIPCHECK(hipMemcpy(b->tile_box_d, tb.data(), sizeof(uint32_t) * tiles, hipMemcpyHostToDevice), "tile table copy");
  HIPCHECK(hipMemcpy(b->boxes_d, b->boxes.data(), sizeof(BoxInfo) * b->boxes.size(), hipMemcpyHostToDevice),
           "box table copy");
  b->ntiles = uint32_t(tiles);
  b->bt = bt;
  return LBM_OK;
}

static void batch_clear_graphs(lbm_batch *b) {
  for (auto &kv : b->gcache) (void)hipGraphExecDestroy(kv.second);
  b->gcache.clear();
}

static lbm_status batch_staging(lbm_batch *b, size_t nd) {
  if (b->staging_doubles >= nd) return LBM_OK;
  if (b->staging) {
    HIPCHECK(hipStreamSynchronize(b->stream), "sync");
    (void)hipFree(b->staging);
    b->staging = nullptr;
    b->staging_doubles = 0;
  }
  hipError_t e = hipMalloc(&b->staging, nd * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(LBM_ENOMEM, "staging allocation failed");
  }
  b->staging_doubles = nd;
  return LBM_OK;
}

static FieldArgs batch_field(const lbm_batch *b, int k, void *base) {
  const BoxInfo &B = b->boxes[k];
  FieldArgs a;
  std::memset(&a, 0, sizeof(a));
  a.buf = static_cast<char *>(base) + size_t(B.off) * b->elem;
  a.L.ps = b->ntot;
  a.L.zs = uint64_t(B.nx) * uint64_t(B.ny);
  a.L.ys = uint32_t(B.nx);
  a.ncells = B.ncells;
  a.nx = B.nx;
  a.ny = B.ny;
  a.nz = B.nz;
  a.tiles_x = (B.nx + FBX - 1) / FBX;
  a.tiles_y = (B.ny + FBY - 1) / FBY;
  return a;
}

static lbm_status batch_launch_field(lbm_batch *b, const void *fn, FieldArgs &a) {
  if (!fn) return fail(LBM_EUNSUPPORTED, "no kernel for this layout");
  void *args[] = {&a};
  HIPCHECK(hipLaunchKernel(fn, field_grid(a, a.nz), dim3(FBX, FBY), args, 0, b->stream), "field kernel launch");
  return LBM_OK;
}

}  // namespace lbm

extern "C" lbm_status lbm_batch_create(const lbm_params *common, int nboxes, const int64_t *dims,
                                       const double *omegas, lbm_batch **out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!common || !dims || !omegas || nboxes < 1) return fail(LBM_EINVAL, "bad batch arguments");
  if (common->stencil == LBM_D2Q9) return fail(LBM_EUNSUPPORTED, "the batched ensemble is three-dimensional");
  if (common->stencil == LBM_D3Q15) return fail(LBM_EUNSUPPORTED, "the batched ensemble runs D3Q19 and D3Q27");
  if (common->streaming != LBM_STREAM_PULL) return fail(LBM_EUNSUPPORTED, "the batched ensemble uses the pull pattern");
  if (common->equilibrium != LBM_EQ_MAXWELLIAN) return fail(LBM_EUNSUPPORTED, "the batched ensemble uses the Maxwellian");
  if (!common->zero_centered) return fail(LBM_EUNSUPPORTED, "the batched ensemble stores zero-centred populations");
  if (common->arithmetic != LBM_ARITH_DEVIATION)
    return fail(LBM_EUNSUPPORTED, "the batched ensemble uses the deviation arithmetic");
  if (common->force[0] != 0.0 || common->force[1] != 0.0 || common->force[2] != 0.0)
    return fail(LBM_EUNSUPPORTED, "the batched ensemble runs without a body force");
  if (common->basis != LBM_BASIS_GRADED) return fail(LBM_EUNSUPPORTED, "the batched ensemble uses the graded basis");
  lbm_batch *b = new lbm_batch();
  b->p = *common;
  b->s = common->stencil;
  b->q = stencil_q(b->s);
  b->d = 3;
  b->space = internal_space(common->space);
  if (const char *env = std::getenv("LBM_BATCH_SWIZZLE")) b->swz = env[0] == '0' ? 0 : 1;
  b->store = common->storage;
  b->elem = storage_bytes(b->store);
  b->nboxes = nboxes;
  std::vector<RelaxHost> rh(nboxes);
  uint64_t off = 0, tiles = 0;
  for (int k = 0; k < nboxes; ++k) {
    lbm_params pk = *common;
    pk.nx = dims[3 * k];
    pk.ny = dims[3 * k + 1];
    pk.nz = dims[3 * k + 2];
    pk.omegas = omegas + size_t(k) * b->q;
    pk.n_omegas = b->q;
    lbm_status s = validate(&pk);
    if (s == LBM_OK) s = relaxation_blocks(b->s, pk.basis, pk.omegas, &rh[k]);
    if (s != LBM_OK) {
      delete b;
      return fail(s, "box " + std::to_string(k) + ": " + g_last_error);
    }
    b->reg = b->reg && rh[k].regularized;
    BoxInfo B;
    B.off = uint32_t(off);
    B.ncells = uint32_t(pk.nx * pk.ny * pk.nz);
    B.tile0 = uint32_t(tiles);
    B.nx = int(pk.nx);
    B.ny = int(pk.ny);
    B.nz = int(pk.nz);
    b->boxes.push_back(B);
    off += B.ncells;
    tiles += (B.ncells + BATCH_THREADS - 1) / BATCH_THREADS;
  }
  if (off * b->elem >= (uint64_t(1) << 32) || tiles >= (uint64_t(1) << 31)) {
    delete b;
    return fail(LBM_EUNSUPPORTED, "one population plane of the ensemble must stay below 4 GiB");
  }
  b->ntot = uint32_t(off);
  b->ntiles = uint32_t(tiles);
  std::vector<uint32_t> tb(b->ntiles);
  for (int k = 0; k < nboxes; ++k) {
    const uint32_t nt = (b->boxes[k].ncells + BATCH_THREADS - 1) / BATCH_THREADS;
    for (uint32_t j = 0; j < nt; ++j) tb[b->boxes[k].tile0 + j] = uint32_t(k);
  }
  auto bail = [&](hipError_t e, const char *what) {
    lbm_batch_destroy(b);
    return hip_fail(e, what);
  };
  hipError_t e;
  const size_t plane_bytes = size_t(b->ntot) * b->elem, buf_bytes = plane_bytes * b->q;
  if (lbm_status sm = check_free_memory(2 * buf_bytes, "population buffer"); sm != LBM_OK) {
    lbm_batch_destroy(b);
    return sm;
  }
  for (int k = 0; k < 2; ++k) {
    e = hipMalloc(&b->buf[k], buf_bytes);
    if (e != hipSuccess) return bail(e, "population buffer allocation");
  }
  if ((e = hipMalloc(&b->boxes_d, sizeof(BoxInfo) * nboxes)) != hipSuccess) return bail(e, "box table");
  if ((e = hipMalloc(&b->tile_box_d, sizeof(uint32_t) * b->ntiles)) != hipSuccess) return bail(e, "tile table");
  b->ntiles_cap = b->ntiles;
  const bool dbl = b->store == F64;
  const size_t rsz = dbl ? sizeof(Relax<double>) : sizeof(Relax<float>);
  if ((e = hipMalloc(&b->relax_d, rsz * nboxes)) != hipSuccess) return bail(e, "relaxation table");
  std::vector<char> rbytes(rsz * nboxes);
  for (int k = 0; k < nboxes; ++k) {
    auto fill = [&](auto *R) {
      using CT = std::remove_reference_t<decltype(R->b6)>;
      for (int j = 0; j < 6; ++j)
        for (int i = 0; i < 6; ++i) R->b2[j][i] = CT(rh[k].b2[j][i]);
      for (int j = 0; j < 7; ++j)
        for (int i = 0; i < 7; ++i) R->b3[j][i] = CT(rh[k].b3[j][i]);
      for (int j = 0; j < 6; ++j)
        for (int i = 0; i < 6; ++i) R->b4[j][i] = CT(rh[k].b4[j][i]);
      for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i) R->b5[j][i] = CT(rh[k].b5[j][i]);
      R->b6 = CT(rh[k].b6);
    };
    if (dbl) fill(reinterpret_cast<Relax<double> *>(rbytes.data()) + k);
    else fill(reinterpret_cast<Relax<float> *>(rbytes.data()) + k);
  }
  if (common->stream) {
    b->stream = static_cast<hipStream_t>(common->stream);
  } else {
    if ((e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)) != hipSuccess) return bail(e, "stream");
    b->own_stream = true;
  }
  if ((e = hipMemcpy(b->boxes_d, b->boxes.data(), sizeof(BoxInfo) * nboxes, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(e, "box table copy");
  if ((e = hipMemcpy(b->tile_box_d, tb.data(), sizeof(uint32_t) * b->ntiles, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(e, "tile table copy");
  if ((e = hipMemcpy(b->relax_d, rbytes.data(), rbytes.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return bail(e, "relaxation table copy");
  *out = b;
  return LBM_OK;
}

extern "C" void lbm_batch_destroy(lbm_batch *b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (auto &kv : b->gcache) (void)hipGraphExecDestroy(kv.second);
  for (int k = 0; k < 2; ++k)
    if (b->buf[k]) (void)hipFree(b->buf[k]);
  if (b->boxes_d) (void)hipFree(b->boxes_d);
  if (b->tile_box_d) (void)hipFree(b->tile_box_d);
  if (b->relax_d) (void)hipFree(b->relax_d);
  if (b->staging) (void)hipFree(b->staging);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

extern "C" lbm_status lbm_batch_init_equilibrium(lbm_batch *b, const double *rho, const double *u) {
  if (!b || !rho || !u) return fail(LBM_EINVAL, "NULL argument");
  const size_t n = b->ntot;
  lbm_status s = batch_staging(b, 4 * n);
  if (s != LBM_OK) return s;
  HIPCHECK(hipMemcpyAsync(b->staging, rho, n * sizeof(double), hipMemcpyDefault, b->stream), "copy rho");
  HIPCHECK(hipMemcpyAsync(b->staging + n, u, 3 * n * sizeof(double), hipMemcpyDefault, b->stream), "copy u");
  b->t = 0;
  b->cur = 0;
  const void *fn = init_fn(b->s, b->store, b->space, MAXWELL, G_SHIFTED);
  for (int k = 0; k < b->nboxes; ++k) {
    FieldArgs a = batch_field(b, k, b->buf[0]);
    a.rho_in = b->staging + b->boxes[k].off;
    a.u_in = b->staging + n + 3 * size_t(b->boxes[k].off);
    s = batch_launch_field(b, fn, a);
    if (s != LBM_OK) return s;
  }
  HIPCHECK(hipStreamSynchronize(b->stream), "init sync");
  return LBM_OK;
}

namespace lbm {
static lbm_status batch_graph_for(lbm_batch *b, int64_t n, hipGraphExec_t *out) {
  auto key = std::make_pair(n, b->cur);
  auto it = b->gcache.find(key);
  if (it == b->gcache.end()) {
    if (b->gcache.size() >= GRAPH_CACHE_MAX) {
      HIPCHECK(hipStreamSynchronize(b->stream), "sync before graph eviction");
      batch_clear_graphs(b);
    }
    const int cur0 = b->cur;
    const int64_t t0 = b->t;
    HIPCHECK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    lbm_status s = LBM_OK;
    for (int64_t k = 0; k < n && s == LBM_OK; ++k) s = batch_one_step(b);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    b->cur = cur0;
    b->t = t0;
    if (s != LBM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    it = b->gcache.emplace(key, ex).first;
  }
  *out = it->second;
  return LBM_OK;
}
}  // namespace lbm

extern "C" lbm_status lbm_batch_step(lbm_batch *b, int64_t n) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  if (n == 0) return LBM_OK;
  if (!b->graphs || n < 2) {
    for (int64_t k = 0; k < n; ++k) {
      lbm_status s = batch_one_step(b);
      if (s != LBM_OK) return s;
    }
    return LBM_OK;
  }
  while (n >= 2) {
    const int64_t m = std::min(n, GRAPH_CHUNK);
    hipGraphExec_t ex = nullptr;
    lbm_status s = batch_graph_for(b, m, &ex);
    if (s != LBM_OK) return s;
    HIPCHECK(hipGraphLaunch(ex, b->stream), "graph launch");
    b->cur ^= int(m & 1);
    b->t += m;
    n -= m;
  }
  return n == 1 ? batch_one_step(b) : LBM_OK;
}

extern "C" lbm_status lbm_batch_graph_prepare(lbm_batch *b, int64_t n) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (n < 2 || !b->graphs) return LBM_OK;
  hipGraphExec_t ex = nullptr;
  lbm_status s = batch_graph_for(b, std::min(n, GRAPH_CHUNK), &ex);
  if (s == LBM_OK && n > GRAPH_CHUNK && n % GRAPH_CHUNK >= 2) s = batch_graph_for(b, n % GRAPH_CHUNK, &ex);
  return s;
}

extern "C" lbm_status lbm_batch_macroscopic(lbm_batch *b, double *rho, double *u) {
  if (!b || !rho || !u) return fail(LBM_EINVAL, "NULL argument");
  const size_t n = b->ntot;
  lbm_status s = batch_staging(b, 4 * n);
  if (s != LBM_OK) return s;
  const void *fn = macro_fn(b->s, b->store, G_SHIFTED);
  for (int k = 0; k < b->nboxes; ++k) {
    FieldArgs a = batch_field(b, k, b->buf[b->cur]);
    a.rho_out = b->staging + b->boxes[k].off;
    a.u_out = b->staging + n + 3 * size_t(b->boxes[k].off);
    s = batch_launch_field(b, fn, a);
    if (s != LBM_OK) return s;
  }
  HIPCHECK(hipMemcpyAsync(rho, b->staging, n * sizeof(double), hipMemcpyDefault, b->stream), "copy rho");
  HIPCHECK(hipMemcpyAsync(u, b->staging + n, 3 * n * sizeof(double), hipMemcpyDefault, b->stream), "copy u");
  HIPCHECK(hipStreamSynchronize(b->stream), "macroscopic sync");
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_get_populations(lbm_batch *b, double *df) {
  if (!b || !df) return fail(LBM_EINVAL, "NULL argument");
  const void *fn = export_fn(b->s, b->store, G_SHIFTED);
  for (int k = 0; k < b->nboxes; ++k) {
    const BoxInfo &B = b->boxes[k];
    lbm_status s = batch_staging(b, size_t(b->q) * B.ncells);
    if (s != LBM_OK) return s;
    FieldArgs a = batch_field(b, k, b->buf[b->cur]);
    a.pop = b->staging;
    a.i0 = 0;
    a.i1 = b->q;
    s = batch_launch_field(b, fn, a);
    if (s != LBM_OK) return s;
    HIPCHECK(hipMemcpyAsync(df + size_t(b->q) * B.off, b->staging, size_t(b->q) * B.ncells * sizeof(double),
                            hipMemcpyDefault, b->stream),
             "copy populations");
    HIPCHECK(hipStreamSynchronize(b->stream), "populations sync");
  }
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_get_box_populations(lbm_batch *b, int k, double *df) {
  if (!b || !df) return fail(LBM_EINVAL, "NULL argument");
  if (k < 0 || k >= b->nboxes) return fail(LBM_EINVAL, "box index out of range");
  const BoxInfo &B = b->boxes[k];
  lbm_status s = batch_staging(b, size_t(b->q) * B.ncells);
  if (s != LBM_OK) return s;
  FieldArgs a = batch_field(b, k, b->buf[b->cur]);
  a.pop = b->staging;
  a.i0 = 0;
  a.i1 = b->q;
  s = batch_launch_field(b, export_fn(b->s, b->store, G_SHIFTED), a);
  if (s != LBM_OK) return s;
  HIPCHECK(hipMemcpyAsync(df, b->staging, size_t(b->q) * B.ncells * sizeof(double), hipMemcpyDefault, b->stream),
           "copy populations");
  HIPCHECK(hipStreamSynchronize(b->stream), "populations sync");
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_synchronize(lbm_batch *b) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  HIPCHECK(hipStreamSynchronize(b->stream), "synchronize");
  return LBM_OK;
}

extern "C" int64_t lbm_batch_cells(const lbm_batch *b) { return b ? int64_t(b->ntot) : -1; }

extern "C" lbm_status lbm_batch_set_graphs(lbm_batch *b, int enable) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  b->graphs = enable != 0;
  return LBM_OK;
}

extern "C" lbm_status lbm_batch_set_launch(lbm_batch *b, int threads, int swizzle, int lds_bytes) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (threads < 64 || threads > BATCH_MAX_THREADS || threads % 64 != 0)
    return fail(LBM_EINVAL, "threads must be a multiple of 64 in [64, 512]");
  if (lds_bytes < 0 || lds_bytes > 65536) return fail(LBM_EINVAL, "lds_bytes must be in [0, 65536]");
  if (threads != b->bt) {
    lbm_status s = batch_build_tiles(b, threads);
    if (s != LBM_OK) return s;
  }
  batch_clear_graphs(b);
  b->swz = swizzle ? 1 : 0;
  b->lds = lds_bytes;
  return b->persistent ? batch_persistent_grid(b) : LBM_OK;
}

extern "C" lbm_status lbm_batch_set_persistent(lbm_batch *b, int enable) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  batch_clear_graphs(b);
  b->persistent = enable != 0;
  return b->persistent ? batch_persistent_grid(b) : LBM_OK;
}

extern "C" int lbm_batch_get_persistent(const lbm_batch *b) { return b && b->persistent ? 1 : 0; }

extern "C" lbm_status lbm_batch_get_launch(const lbm_batch *b, int *threads, int *swizzle, int *lds_bytes) {
  if (!b || !threads || !swizzle || !lds_bytes) return fail(LBM_EINVAL, "NULL argument");
  *threads = b->bt;
  *swizzle = b->swz;
  *lds_bytes = b->lds;
  return LBM_OK;
}

// Times one sweep (src -> dst, the state and the step counter untouched) for every tile size,
// XCD order and LDS reserve, and keeps the fastest.
extern "C" lbm_status lbm_batch_autotune(lbm_batch *b) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  const int cur0 = b->cur;
  const int64_t t0 = b->t;
  const int bt0 = b->bt, swz0 = b->swz, lds0 = b->lds;
  const bool pers0 = b->persistent;
  EventPair ev;
  HIPCHECK(ev.create(), "event");
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  const int reps = 5;
  double best = 1e300;
  int bb[4] = {bt0, swz0, lds0, pers0 ? 1 : 0};
  lbm_status st = LBM_OK;
  for (int bt : {64, 128, 256, 512}) {
    st = batch_build_tiles(b, bt);
    for (int swz : {0, 1})
      for (int lds : {0, 16384, 20480, 26624, 32768, 40960, 53248, 65536})
        for (int pers : {0, 1}) {
          if (st != LBM_OK) break;
          b->swz = swz;
          b->lds = lds;
          b->persistent = pers != 0;
          if (pers) st = batch_persistent_grid(b);
          for (int r = 0; r < reps + 1 && st == LBM_OK; ++r) {
            if (r == 1) (void)hipEventRecord(e0, b->stream);
            b->cur = cur0;
            b->t = t0;
            st = batch_one_step(b);
          }
          (void)hipEventRecord(e1, b->stream);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (st != LBM_OK) break;
          if (std::getenv("LBM_AUTOTUNE_VERBOSE"))
            std::fprintf(stderr, "[lbm batch autotune] threads %d swizzle %d lds %d persistent %d: %.4f ms/step\n", bt,
                         swz, lds, pers, ms / reps);
          if (ms < best) {
            best = ms;
            bb[0] = bt;
            bb[1] = swz;
            bb[2] = lds;
            bb[3] = pers;
          }
        }
    if (st != LBM_OK) break;
  }
  b->cur = cur0;
  b->t = t0;
  lbm_status s2 = batch_build_tiles(b, st == LBM_OK ? bb[0] : bt0);
  b->swz = st == LBM_OK ? bb[1] : swz0;
  b->lds = st == LBM_OK ? bb[2] : lds0;
  b->persistent = st == LBM_OK ? bb[3] != 0 : pers0;
  if (s2 == LBM_OK && b->persistent) s2 = batch_persistent_grid(b);
  batch_clear_graphs(b);
  return st != LBM_OK ? st : s2;
}

extern "C" lbm_status lbm_batch_time_steps(lbm_batch *b, int64_t n, double *ms) {
  if (!b || !ms) return fail(LBM_EINVAL, "NULL argument");
  EventPair ev;
  HIPCHECK(ev.create(), "event");
  HIPCHECK(hipEventRecord(ev.e0, b->stream), "event record");
  lbm_status s = lbm_batch_step(b, n);
  HIPCHECK(hipEventRecord(ev.e1, b->stream), "event record");
  float f = 0.f;
  HIPCHECK(ev.elapsed(&f), "elapsed");
  *ms = double(f);
  return s;
}
