// Host-side method description shared by the library's translation units.
#pragma once

#include <stdint.h>

#include <string>

#include "../../include/lbm.h"

namespace lbm {

// B = I - P^-1 S P per order (rows/cols in the device's order lists), FP64
struct RelaxHost {
  double b2[6][6];
  double b3[7][7];
  double b4[6][6];
  double b5[3][3];
  double b6;
  // cross-order blocks of a basis whose polynomials mix orders (the orthogonal bases):
  // dm*_3 += c31 dm_1, dm*_4 += c42 dm_2, dm*_5 += c53 dm_3 + c51 dm_1,
  // dm*_6 += c62 . dm_2 + c64 . dm_4 (pre-relaxation deviations; the first-order deviations
  // are nonzero only with a body force, the zeroth-order ones never)
  double c31[7][3];
  double c42[6][6];
  double c51[3][3];
  double c53[3][7];
  double c62[6];
  double c64[6];
  bool cross;        // some cross-order block between orders >= 2 is nonzero
  bool cross1;       // some block from order 1 (c31, c51) is nonzero: acts only with a force
  bool regularized;  // every block of order >= 3 vanishes (all those rates equal 1)
};

extern thread_local std::string g_last_error;
lbm_status fail(lbm_status s, const std::string &msg);
int stencil_q(int s);
int stencil_d(int s);
size_t storage_bytes(int st);
int resolve_eq_form(const lbm_params *p);
// kernel-side identifiers (the device headers' SpaceId::SRT and LiteralForm)
constexpr int kSpaceSrt = 4;
constexpr int kLitA = 0, kLitB = 1, kLitC = 2;
// kernel space id of a public lbm_space
int internal_space(int public_space);
// LITERAL arithmetic: which form of sec. 2.2 the parameter set selects (kLitA/B/C)
int literal_form(const lbm_params *p);
size_t plane_elems(const lbm_params *p);
int resolve_layout(const lbm_params *p);
void storage_strides(const lbm_params *p, uint64_t *ps, uint64_t *zs, uint64_t *ys, uint64_t *elems);
constexpr size_t kDefaultPlanePadBytes = 0;
lbm_status validate(const lbm_params *p);
lbm_status relaxation_blocks(int s, int basis, const double *omegas, RelaxHost *out);

}  // namespace lbm
