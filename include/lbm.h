/*
 * lbm.h -- C ABI of the MI355X (gfx950) zero-centred multiple-relaxation-time lattice
 * Boltzmann library.
 *
 * The operations follow Hennig, Holzer, Ruede, "Advanced Automatic Code Generation for
 * Multiple Relaxation-Time Lattice Boltzmann Methods" (arXiv 2211.02435):
 *   - a method is a stencil, a storage format, a collision space with a polynomial basis,
 *     one relaxation rate per basis polynomial and an equilibrium (sec. 3, configuration
 *     space of the modelling front-end);
 *   - one time step is the fused collide-and-stream update of eq. LbUpdateScheme (sec. 2.1)
 *     with the collision of eq. MrtUpdateGeneralDeviationOnly (raw or central moments with
 *     the delta-equilibrium) or eq. MrtUpdateAbsoluteFromZeroCentered (any space with the
 *     absolute equilibrium), sec. 2.2, on zero-centred populations df = f - f0 (sec. 2.1);
 *   - the collision-space transforms are the raw-moment Chimera transform (eq.
 *     RawMomentChimeraTransform, sec. 4.1.1), the binomial Chimera transform between raw
 *     and central moments (sec. 4.2) and the central-moment / cumulant relation of
 *     eq. CumulantAndCentralMomentGenFuncs (sec. 4.2.1).
 *
 * Conventions (the paper fixes only xi_0 = 0):
 *   Velocity order, opposite pairs adjacent (opp(i) = i+1 for odd i):
 *     D2Q9 : (0,0) (1,0) (-1,0) (0,1) (0,-1) (1,1) (-1,-1) (1,-1) (-1,1)
 *     D3Q27: (0,0,0); (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1);
 *            (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
 *            (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1);
 *            (1,1,1) (-1,-1,-1) (1,1,-1) (-1,-1,1) (1,-1,1) (-1,1,-1) (-1,1,1) (1,-1,-1)
 *     D3Q19: the first 19 velocities of D3Q27.
 *     D3Q15: the first 7 velocities of D3Q27 and its 8 corners, in D3Q27's order.
 *   Weights (background f0 for the Maxwellian equilibrium, f0 = M^-1 m0 = w, sec. 2.4):
 *     D2Q9 4/9 1/9 1/36; D3Q19 1/3 1/18 1/36; D3Q27 8/27 2/27 1/54 1/216; D3Q15 2/9 1/9
 *     (faces) 1/72 (corners).  c_s^2 = 1/3,
 *     rho0 = 1.  For the shallow-water equilibrium f0 = f^eq(h = 1, u = 0).
 *   Polynomial basis, one relaxation rate per entry of `omegas`, in this order
 *   (graded: every polynomial is homogeneous in one order):
 *     D2Q9 (the basis of the shallow-water listing, sec. 5.2):
 *       1, x, y, xy, x2-y2, x2+y2, xy2, x2y, x2y2
 *     D3Q19: 1, x, y, z, xy, xz, yz, x2-y2, x2-z2, x2+y2+z2,
 *            xy2+xz2, xy2-xz2, x2y+yz2, x2y-yz2, x2z+y2z, x2z-y2z,
 *            x2y2-2x2z2+y2z2, x2y2+x2z2-2y2z2, x2y2+x2z2+y2z2
 *     D3Q27: the first 16 of D3Q19, xyz, the three fourth-order combinations of D3Q19,
 *            x2yz, xy2z, xyz2, xy2z2, x2yz2, x2y2z, x2y2z2
 *     D3Q15: 1, x, y, z, xy, xz, yz, x2-y2, x2-z2, x2+y2+z2, xyz, xy2, x2y, x2z, x2y2, where
 *            xy2 stands for its class on the lattice (xy2 = xz2 = xy2z2 there), x2y for
 *            (x2y, yz2, x2yz2), x2z for (x2z, y2z, x2y2z) and x2y2 for the corner indicator
 *            (x2y2 = x2z2 = y2z2 = x2y2z2).  In raw-moment space and SRT D3Q15 takes the
 *            second-order polynomial equilibrium (its raw classes cannot carry the
 *            Maxwellian's raw moments); in central-moment and cumulant space the
 *            Maxwellian's central moments are imposed on these 15 monomials, a set closed
 *            under lowering exponents and hence under the binomial shift.
 *     Rates of the conserved polynomials 1, x, y, z are ignored.
 *   Equilibria: LBM_EQ_MAXWELLIAN is the continuous Maxwellian of sec. 2.4; its raw moments
 *     are truncated at second order in u (sec. 4.3), its central moments and cumulants are
 *     used exactly (they do not depend on u).  LBM_EQ_SHALLOW_WATER is the discrete D2Q9
 *     equilibrium of Zhou (sec. 5.2) with the listing's -u.u/6 term; `gravity` is g.
 *
 * Memory layout of every field argument: SoA, x fastest (the device population buffers use
 * the same order with a padded plane stride, see lbm_required_bytes).
 *   cell(x, y, z) = (z * ny + y) * nx + x, ncells = nx * ny * nz
 *   populations  df[i * ncells + cell]          (canonical pre-collision df(t), FP64)
 *   density      rho[cell]   (water height h for the shallow-water equilibrium)
 *   velocity     u[d * ncells + cell], d = 0 (x), 1 (y), 2 (z); D2Q9 ignores/zeroes d = 2
 * Host or device pointers are accepted wherever a field pointer is taken (detected with
 * hipPointerGetAttributes).  Pointers are borrowed for the duration of the call only.
 *
 * Time convention: df(0) = f^eq(rho0, u0) - f0; lbm_step(1) collides, then streams, so that
 * after t steps the readers (macroscopic, get_populations, diagnostics) report df(t).
 *
 * Errors: every call returns an lbm_status; the message of the last failure of the calling
 * thread is returned by lbm_last_error().  No call aborts the process.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,        /* invalid argument: enum out of range, dims < 1, n_omegas != q, ...  */
  LBM_EUNSUPPORTED = -2,  /* inadmissible combination (sec. 3) or not implemented               */
  LBM_ENOMEM = -3,        /* device allocation failed or caller buffer too small               */
  LBM_EDEVICE = -4,       /* a HIP runtime error; lbm_last_error() holds the HIP message       */
  LBM_ENONFINITE = -5     /* lbm_diagnostics found NaN or Inf populations                      */
} lbm_status;

typedef enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1, LBM_D3Q27 = 2, LBM_D3Q15 = 3 } lbm_stencil;
/* SRT: the single-relaxation-time method in population space (eq. MrtUpdateGeneral with the
 * identity transform and S = omega I, the SRT row of the method table of sec. 4.3); its
 * equilibrium is the second-order polynomial f_eq_i = w_i rho (1 + 3 xi.u + 9/2 (xi.u)^2
 * - 3/2 u.u), and every rate of a non-conserved polynomial must be the same omega. */
typedef enum { LBM_SPACE_RAW = 0, LBM_SPACE_CENTRAL = 1, LBM_SPACE_CUMULANT = 2, LBM_SPACE_SRT = 3 } lbm_space;
/* LBM_EQ_SHALLOW_WATER_CONTINUOUS: Venturi's shallow-water equilibrium, the continuous
 * Maxwellian of sec. 2.4 with density h and squared speed of sound c^2 = g h / 2 (sec. 5.2),
 * used exactly in central-moment or cumulant space; background f0 = f^eq(h = 1, u = 0). */
typedef enum {
  LBM_EQ_MAXWELLIAN = 0,
  LBM_EQ_SHALLOW_WATER = 1,
  LBM_EQ_SHALLOW_WATER_CONTINUOUS = 2
} lbm_equilibrium;
/* DEFAULT resolves to DELTA for raw and central moments and SRT with the Maxwellian, to
 * ABSOLUTE for cumulants and for the shallow-water equilibrium. */
typedef enum { LBM_EQFORM_DEFAULT = 0, LBM_EQFORM_ABSOLUTE = 1, LBM_EQFORM_DELTA = 2 } lbm_eq_form;
/* Storage precision of the populations.  Compute precision is FP64 for F64 storage and FP32
 * for F32 and F16 storage.  Initialisation and every reader compute in FP64. */
typedef enum { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_F16 = 2 } lbm_storage;
/* PULL: two arrays, each step gathers f_i(x) from x - xi_i.  PUSH: two arrays, each step
 * reads the cell's own populations and scatters f*_i to x + xi_i.  AA: one array, in place
 * (even steps read and write the cell's own slots, odd steps read from x - xi_i and write to
 * x + xi_i); sec. 4.4. */
/* ESOTERIC_PULL: one array, in place (sec. 4.4): every step a cell touches its own slots and
 * the neighbours x + xi of one direction of each opposite pair (the odd indices); population i
 * of an odd direction (and the rest) is kept at the cell, that of an even direction at
 * x - xi, in slot opp(i) after an even number of steps and in slot i after an odd number.
 * ESOTERIC_TWIST: one array, in place (sec. 4.4): every step a cell touches the nodes
 * x + {0,1}^3 only; population i is kept at x + (-xi)^+ (componentwise positive part), in
 * slot i after an even number of steps and in slot opp(i) after an odd number.  Readers,
 * writers and lbm_set_time translate every layout to and from the canonical df(t). */
typedef enum {
  LBM_STREAM_PULL = 0,
  LBM_STREAM_AA = 1,
  LBM_STREAM_ESOTERIC_PULL = 2,
  LBM_STREAM_ESOTERIC_TWIST = 3,
  LBM_STREAM_PUSH = 4
} lbm_streaming;

/* How the collision's arithmetic is organised.  DEVIATION: every intermediate is a deviation
 * from the background (raw, central and cumulant moments of df, the equilibrium deviation
 * expanded so that no background value is subtracted), whatever the storage format and
 * eq_form; in exact arithmetic it equals each admissible form of sec. 2.2.  LITERAL: the form
 * is evaluated as written, for the round-off study of sec. 5.1: absolute storage ->
 * eq. MrtUpdateGeneral on absolute populations and moments; zero-centred storage with the
 * delta-equilibrium -> eq. MrtUpdateGeneralDeviationOnly with dq_eq = q_eq - T(f0) formed by
 * subtraction; zero-centred storage with the absolute equilibrium ->
 * eq. MrtUpdateAbsoluteFromZeroCentered (q = T(df + f0), df* = T^-1(q*) - f0).  LITERAL
 * covers D2Q9 and D3Q27, F64 and F32 storage, pull streaming, the Maxwellian equilibrium. */
typedef enum { LBM_ARITH_DEVIATION = 0, LBM_ARITH_LITERAL = 1 } lbm_arithmetic;

/* Source-term model of a body force (sec. 2.1 cites both): GUO (Guo, Zheng, Shi):
 * S_i = w_i [(xi_i - u) / cs2 + (xi_i . u) xi_i / cs4] . F;  HE (He, Shan, Doolen):
 * S_i = (xi_i - u) . F f_eq_i / (rho cs2) with the method's equilibrium populations.  Both
 * shift the equilibrium velocity to u = (j + F/2) / rho and add (I - S/2) T(S). */
typedef enum { LBM_FORCE_GUO = 0, LBM_FORCE_HE = 1 } lbm_force_model;

/* Polynomial basis in which raw moments are relaxed (sec. 2.3.1, Table 1).  GRADED: the basis
 * listed above, every polynomial homogeneous in one order.  WEIGHTED_ORTHOGONAL (WO-MRT): the
 * Gram-Schmidt orthogonalisation of the graded basis, in its order, under the inner product
 * <a, b> = sum_i w_i a(xi_i) b(xi_i); omegas[k] is the rate of the k-th orthogonalised
 * polynomial.  Its polynomials mix orders, so the relaxation couples a moment to lower orders
 * of the same parity.  ORTHOGONAL (O-MRT): the same with the plain sum over the velocities
 * (on D2Q9 the polynomials of Lallemand and Luo).  The orthogonal bases need the raw-moment
 * space, the Maxwellian equilibrium and D2Q9, D3Q19 or D3Q27 (LBM_EUNSUPPORTED otherwise); with every rate equal to 1 they equal GRADED.  With a body
 * force the first-order deviations (-F/2) also reach orders 3 and 5. */
typedef enum { LBM_BASIS_GRADED = 0, LBM_BASIS_WEIGHTED_ORTHOGONAL = 1, LBM_BASIS_ORTHOGONAL = 2 } lbm_basis;

/* Device layout of the populations (x fastest in both).  PLANES: one plane per population,
 * [q][z][y][x] with a padded plane stride.  ROWS: the q populations of one row side by side,
 * [z][y][q][x], so the rows a block reads and writes are contiguous.  AUTO: ROWS (the faster
 * layout measured on MI355X for every storage type and streaming pattern), or PLANES where one
 * z-plane of the ROWS layout would reach 4 GiB. */
typedef enum { LBM_LAYOUT_AUTO = 0, LBM_LAYOUT_PLANES = 1, LBM_LAYOUT_ROWS = 2 } lbm_layout;

typedef struct {
  int stencil;            /* lbm_stencil                                                      */
  int space;              /* lbm_space                                                        */
  int equilibrium;        /* lbm_equilibrium                                                  */
  int eq_form;            /* lbm_eq_form                                                      */
  int zero_centered;      /* 1: store df = f - f0 (sec. 2.1); 0: store absolute f (Maxwellian) */
  const double *omegas;   /* host array of n_omegas rates, basis order above, each in [0, 2]  */
  int n_omegas;           /* == q                                                             */
  double gravity;         /* g > 0 for the shallow-water equilibria, ignored otherwise        */
  int64_t nx, ny, nz;     /* lattice size; nz == 1 for D2Q9                                   */
  int periodic[3];        /* must be {1, 1, 1}                                                */
  int storage;            /* lbm_storage                                                      */
  int streaming;          /* lbm_streaming                                                    */
  void *buffers[2];       /* optional caller-owned device buffers (e.g. torch allocations);   */
                          /* LBM_EINVAL from lbm_create if one is not device memory          */
  size_t buffer_bytes;    /* each >= lbm_required_bytes / nbuffers; NULL -> library allocates */
  void *stream;           /* hipStream_t to run on; NULL -> the library creates its own       */
  int layout;             /* lbm_layout of the device population buffers                      */
  int arithmetic;         /* lbm_arithmetic of the collision                                  */
  double force[3];        /* constant body force per cell and step (lattice units);           */
                          /* {0, 0, 0} for none.  See lbm_set_force_field.                    */
  int force_model;        /* lbm_force_model of any body force                                */
  int basis;              /* lbm_basis of the raw-moment relaxation                           */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Fill *p with defaults: D3Q27, cumulant, Maxwellian, DEFAULT form, zero-centred, FP32, pull,
 * periodic, 1x1x1, no rates, AUTO layout, DEVIATION arithmetic, no force (Guo's model),
 * GRADED basis.  Always succeeds for non-NULL p. */
lbm_status lbm_params_default(lbm_params *p);

/* Validate a parameter set without touching any device (pure host code).
 * LBM_EINVAL for bad enums, dims < 1, n_omegas != q, NULL omegas, non-finite or out-of-range
 * rates, gravity <= 0 with the shallow-water equilibrium; LBM_EUNSUPPORTED for boxes of 2^32
 * cells or more (32-bit natural cell indices) or with a z-plane of population storage of
 * 4 GiB or more (32-bit lane offsets).  LBM_EUNSUPPORTED for the
 * restrictions of sec. 3 (delta-equilibrium needs zero-centred storage; the cumulant space
 * admits no delta-equilibrium), absolute storage with the shallow-water equilibrium, D2Q9 with
 * nz != 1, the shallow-water equilibria on a 3-D stencil, Zhou's in cumulant space, Venturi's
 * outside central and cumulant space, non-periodic
 * axes, SRT with unequal rates (EINVAL) or the shallow-water equilibrium, LITERAL arithmetic
 * outside D2Q9/D3Q27, pull, Maxwellian, a body force with LITERAL arithmetic or a
 * shallow-water equilibrium, D3Q15 with another equilibrium or LITERAL arithmetic, and the
 * orthogonal bases outside their domain (lbm_basis).
 * Absolute storage keeps f = df + w in the buffers (the "absolute" storage format of the
 * paper, used for the round-off plateau study of sec. 5.1).  With DEVIATION arithmetic every
 * sweep subtracts w after loading and adds it back before storing, so only the storage
 * rounds f; with LITERAL arithmetic the whole collision runs on absolute values. */
lbm_status lbm_validate(const lbm_params *p);

/* Bytes of device population storage the parameter set needs in total (both arrays for
 * pull and push, one for the in-place patterns).  PLANES: nbuffers * q * plane * sizeof(storage), the plane stride being
 * ncells rounded up to 256 bytes plus a padding that staggers the q planes across HBM
 * channels (environment variable LBM_PLANE_PAD_BYTES overrides the padding).  ROWS:
 * nbuffers * nz * ny * q * nxp * sizeof(storage), nxp = nx rounded up to 256 bytes.
 * Pure host code. */
lbm_status lbm_required_bytes(const lbm_params *p, size_t *bytes);

/* Create a context: validate, derive the relaxation matrix in monomial form, allocate or
 * attach device buffers, pick the launch shape.  *out is NULL on failure.  LBM_ENOMEM when
 * the buffers the library allocates exceed the free device memory (checked with
 * hipMemGetInfo before any allocation is attempted) or a caller buffer is too small. */
lbm_status lbm_create(const lbm_params *p, lbm_ctx **out);
void lbm_destroy(lbm_ctx *ctx);

/* Initialise df(0) = f^eq(rho, u) - f0 from FP64 fields (sec. 2.4); resets the step counter.
 * rho: ncells values; u: 3 * ncells values (d = 2 ignored for D2Q9).  Asynchronous on the
 * context stream when both pointers are device pointers, synchronous otherwise. */
lbm_status lbm_init_equilibrium(lbm_ctx *ctx, const double *rho, const double *u);

/* Advance n >= 0 time steps (fused collide + stream).  Asynchronous on the context stream.
 * With graphs enabled (default) the launches are recorded once into hipGraphs of at most 256
 * steps per (length, buffer parity) and replayed: n / 256 replays of the 256-step graph, then
 * a graph of the remainder (a single remaining step runs directly).  At most 8 graphs are
 * kept per context; recording another one first drops them all. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n);

/* Record (without running) the hipGraphs that the next lbm_step(n) will replay, so that the
 * recording cost stays out of a timed region.  No effect for n < 2 or with graphs off. */
lbm_status lbm_graph_prepare(lbm_ctx *ctx, int64_t n);

/* Body force field (sec. 2.1 source term, eq. MrtUpdateGeneral's q^F) with the model of
 * params.force_model (Guo's by default):
 * F[d * ncells + cell], d = 0..2, FP64, host or device pointer, copied (in the compute
 * precision) and added to the constant params.force in every following step; NULL removes
 * it.  With a force the equilibrium velocity is u = (j + F/2) / rho, the source's moments in
 * the collision space (raw moments, or central moments for the central and cumulant spaces;
 * the populations themselves for SRT) are added weighted by (I - S/2), every cell gains F of
 * momentum per step, and lbm_macroscopic reports that u.  Forced steps use the general
 * (non-regularized) kernels; not with LITERAL arithmetic, the shallow-water equilibria, the
 * MFMA ablation or the batched ensemble (LBM_EUNSUPPORTED).  Synchronous. */
lbm_status lbm_set_force_field(lbm_ctx *ctx, const double *F);

/* Density (or h) and velocity of df(t), FP64, synchronous. */
lbm_status lbm_macroscopic(lbm_ctx *ctx, double *rho, double *u);

/* Canonical df(t) in natural layout, FP64 (export / import for checks and checkpoints).
 * set_populations narrows to the storage precision and keeps the step counter. */
lbm_status lbm_get_populations(lbm_ctx *ctx, double *df);
lbm_status lbm_set_populations(lbm_ctx *ctx, const double *df);

/* FP64 reductions over df(t): out = {sum drho, sum jx, sum jy, sum jz,
 * sum rho |u|^2 / 2 with u = j / rho, number of non-finite populations}.  Deterministic (wave
 * butterflies and block sums in a fixed order).
 * Returns LBM_ENONFINITE when out[5] > 0 (out is still filled).  Synchronous. */
lbm_status lbm_diagnostics(lbm_ctx *ctx, double out[6]);

/* Allocation-free variant of lbm_diagnostics, for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * reductions and the same results as lbm_diagnostics, but the per-block partial sums go to a
 * static device array of LBM_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it
 * runs on until the process ends; the call allocates nothing.
 * out: 6 doubles.  Device memory: the two reduction kernels are queued on the context stream
 * and the call returns without synchronising (out[5] carries the non-finite count; no
 * LBM_ENONFINITE).  Host memory: the call synchronises and returns LBM_ENONFINITE like
 * lbm_diagnostics.
 * The array is shared by every call on one GPU and keeps the last call's contents: calls that
 * overlap on one GPU (other streams, other threads, other contexts) race and must be ordered
 * by the caller.  The context's device must be current (LBM_EINVAL otherwise).
 * LBM_EUNSUPPORTED if the reduction would need more than LBM_NOALLOC_SCRATCH_BYTES (it needs
 * 48 bytes per reduction block, at most 2048 blocks, plus 48). */
#define LBM_NOALLOC_SCRATCH_BYTES (128 * 1024)
lbm_status lbm_diagnostics_noalloc(lbm_ctx *ctx, double *out);
/* Wait for all work queued on the context stream. */
lbm_status lbm_synchronize(lbm_ctx *ctx);

/* Steps taken since the last init (or as set by lbm_set_time). */
int64_t lbm_time(const lbm_ctx *ctx);
/* Set the step counter (checkpoint restore: set_populations, then set_time). */
lbm_status lbm_set_time(lbm_ctx *ctx, int64_t t);

/* Launch shape of the sweep: block of bx * by threads covering bx cells along x and by rows
 * along y; xcd_swizzle != 0 maps consecutive tiles to the same XCD.  bx * by must be a
 * multiple of 64 and <= 512. */
lbm_status lbm_set_launch(lbm_ctx *ctx, int bx, int by, int xcd_swizzle);
lbm_status lbm_get_launch(const lbm_ctx *ctx, int *bx, int *by, int *xcd_swizzle);

/* Vectorised sweep: each lane owns V x-adjacent cells (V = 2 for F64/F32, 4 for F16) and reads
 * each population row segment with one aligned vector load, the x +- 1 neighbours coming from
 * the adjacent lane (wave shift).  Needs nx to be a multiple of bx * V (LBM_EUNSUPPORTED
 * otherwise); AA odd steps use the per-cell kernel (or the LDS-shifted one, lbm_set_staged).
 * Off by default; lbm_autotune
 * considers it. */
lbm_status lbm_set_vectorized(lbm_ctx *ctx, int enable);
int lbm_get_vectorized(const lbm_ctx *ctx);
/* LDS variants of the streaming patterns of sec. 4.4 (eq. LbUpdateScheme).
 * Pull: the LDS-staged sweep.  Each block of bx x 1 threads (bx = 128 or 256) owns bx
 * consecutive cells of one row; it first copies the q source row segments it gathers from
 * (cells x0 - E .. x0 + bx + E - 1 of population i in row (y - cy, z - cz), E elements per
 * 16-byte chunk) from HBM into LDS with 16-byte global-to-LDS loads, then each thread reads its
 * q values from LDS, collides and stores.  Needs by = 1, bx in {128, 256}, nx a multiple of bx
 * and 16-byte aligned population rows.
 * AA: the odd step (which writes slot i at x + xi) puts the post-collision values of the
 * populations with cx != 0 into LDS and stores each row segment of the block aligned, the
 * value of the cell one to the left or right on every position; only the two block ends write
 * single elements.  Needs at most 256 threads per block and nx a multiple of bx.  Even steps
 * use the per-cell kernel.
 * LBM_EUNSUPPORTED for other shapes or patterns; a later lbm_set_launch with a shape the
 * variant cannot run turns it off.  The forced, literal, orthogonal-basis and MFMA kernels
 * ignore it.  Off by default; lbm_autotune considers it.  Results equal the register
 * kernels' bit for bit. */
lbm_status lbm_set_staged(lbm_ctx *ctx, int enable);
int lbm_get_staged(const lbm_ctx *ctx);

/* Collision-space transform of the sweep.  CHIMERA (default): the raw-moment Chimera passes
 * of sec. 4.1.1 in registers.  DENSE_MFMA (measured ablation): m = M df and df* = M^-1 dm* as
 * dense 27 x 27 products over the 64 cells of a wave on the matrix cores, staged through
 * LDS; D3Q27, pull, Maxwellian equilibrium, blocks of 64..256 threads (LBM_EUNSUPPORTED
 * otherwise; a later lbm_set_launch with more threads reverts to CHIMERA). */
typedef enum { LBM_TRANSFORM_CHIMERA = 0, LBM_TRANSFORM_DENSE_MFMA = 1 } lbm_transform;
lbm_status lbm_set_transform(lbm_ctx *ctx, int transform);
int lbm_get_transform(const lbm_ctx *ctx);

/* The layout the context's buffers use (LBM_LAYOUT_PLANES or LBM_LAYOUT_ROWS; AUTO resolved),
 * or -1 for a NULL context. */
int lbm_get_layout(const lbm_ctx *ctx);

/* Dynamic LDS reserved by every sweep block (0 .. 65536 bytes; the register sweeps use none,
 * the LDS-staged sweep takes the larger of the reserve and its own image): caps the resident
 * blocks per CU (160 KB of LDS each), i.e. the number of waves streaming concurrently.  0 by
 * default; lbm_autotune considers it. */
lbm_status lbm_set_lds_reserve(lbm_ctx *ctx, int bytes);
int lbm_get_lds_reserve(const lbm_ctx *ctx);

/* Time candidate launch shapes (block shape, XCD swizzle, per-cell, vectorised or LDS-staged
 * kernel, then the LDS reserve of the best shape of each block size) on
 * the context's own buffers (state is left unchanged) and keep the fastest; results are
 * cached per (method, precision, pattern, layout, size, transform) in the JSON file named by
 * LBM_AUTOTUNE_CACHE, if set.  With the MFMA transform only blocks of at most 256 threads,
 * the per-cell kernel and no LDS reserve are considered.  Every return path restores the
 * state, the step counter and (on failure) the previous launch. */
lbm_status lbm_autotune(lbm_ctx *ctx);

/* Enable (1) or disable (0) hipGraph recording in lbm_step. */
lbm_status lbm_set_graphs(lbm_ctx *ctx, int enable);

/* Device pointer of population buffer k (0 or 1) and the buffer holding the state that the
 * next sweep reads; for measurement and checks. */
lbm_status lbm_buffer(const lbm_ctx *ctx, int k, void **ptr, size_t *bytes);

/* Time n sweeps with HIP events recorded on the context stream; *ms = elapsed milliseconds. */
lbm_status lbm_time_steps(lbm_ctx *ctx, int64_t n, double *ms);

/* Message of the calling thread's last failure ("" if none). */
const char *lbm_last_error(void);

/* Library version string. */
const char *lbm_version(void);

/* --------------------------------------------------------------------------------------
 * Batched ensemble: many independent periodic boxes of one method family, each with its
 * own size and relaxation rates, advanced by one launch per time step over a tile list of
 * all boxes.  Boxes are stored back to back (box b starts at cell offset sum_{c<b} ncells_c).
 * Field arguments are the per-box fields concatenated in box order.
 * -------------------------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

/* common: stencil, space, equilibrium, eq_form, storage, streaming (pull only), stream;
 * its dims, omegas and buffers are ignored.  dims: nboxes * 3 (nx, ny, nz);
 * omegas: nboxes * q rates.  3-D stencils only.  LBM_ENOMEM when the two population arrays
 * exceed the free device memory (checked before allocating). */
lbm_status lbm_batch_create(const lbm_params *common, int nboxes, const int64_t *dims,
                            const double *omegas, lbm_batch **out);
void lbm_batch_destroy(lbm_batch *b);
lbm_status lbm_batch_init_equilibrium(lbm_batch *b, const double *rho, const double *u);
/* n >= 0 steps of every box, one launch per step; graphs as for lbm_step (chunks of at most
 * 256 steps, at most 8 graphs kept).  Asynchronous on the batch stream. */
lbm_status lbm_batch_step(lbm_batch *b, int64_t n);
lbm_status lbm_batch_graph_prepare(lbm_batch *b, int64_t n);
lbm_status lbm_batch_macroscopic(lbm_batch *b, double *rho, double *u);
lbm_status lbm_batch_get_populations(lbm_batch *b, double *df);
/* df(t) of box k alone, natural layout df[i * ncells_k + cell] (q * ncells_k doubles). */
lbm_status lbm_batch_get_box_populations(lbm_batch *b, int k, double *df);
lbm_status lbm_batch_synchronize(lbm_batch *b);
int64_t lbm_batch_cells(const lbm_batch *b);
lbm_status lbm_batch_set_graphs(lbm_batch *b, int enable);
lbm_status lbm_batch_time_steps(lbm_batch *b, int64_t n, double *ms);
/* Launch shape of the ensemble sweep: `threads` cells per tile (= threads per block, a
 * multiple of 64 in [64, 512]; default 256), tiles taken in XCD order (swizzle != 0, default)
 * and `lds_bytes` of dynamic LDS reserved per block (0..65536; caps the resident blocks per
 * CU).  Results do not depend on it.  Rebuilds the tile table; synchronous.  LBM_EINVAL for
 * values out of range. */
lbm_status lbm_batch_set_launch(lbm_batch *b, int threads, int swizzle, int lds_bytes);
lbm_status lbm_batch_get_launch(const lbm_batch *b, int *threads, int *swizzle, int *lds_bytes);
/* Grid form of the ensemble sweep: 0 (default) one block per tile; 1 persistent, a grid of as
 * many blocks as the device holds at once for the current tile size and LDS reserve (a multiple
 * of 8), each block striding over the tile list (in XCD order with the swizzle).  Results do
 * not depend on it.  The grid follows later lbm_batch_set_launch calls. */
lbm_status lbm_batch_set_persistent(lbm_batch *b, int enable);
int lbm_batch_get_persistent(const lbm_batch *b);
/* Times one sweep for every tile size in {64, 128, 256, 512}, both tile orders, the LDS
 * reserves {0, 16, 20, 26, 32, 40, 52, 64} KiB and both grid forms, and keeps the fastest.  The state and the step counter
 * are left unchanged (each timed sweep writes only the other buffer).  Synchronous. */
lbm_status lbm_batch_autotune(lbm_batch *b);

/* --------------------------------------------------------------------------------------
 * Measurement helpers
 * -------------------------------------------------------------------------------------- */
/* Plain device copy of `bytes` bytes (16-byte vector loads and stores) repeated `reps` times,
 * timed with HIP events; the practical HBM ceiling beside the sweep. */
lbm_status lbm_copy_bandwidth(void *dst, const void *src, size_t bytes, int reps, void *stream,
                              double *ms);

/* Test hook: streaming only (the collision replaced by the identity), for checking the
 * integer index maps of the pull and AA patterns bit for bit. */
lbm_status lbm_debug_stream_only(lbm_ctx *ctx, int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
