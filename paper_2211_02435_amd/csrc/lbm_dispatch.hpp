// Kernel lookup: each translation unit instantiates the kernels of one (stencil, storage)
// pair and exports them through these tables; the host library launches by pointer.
#pragma once

namespace lbm {

template <int S, int STORE>
struct KTable {
  static const void *sweep(int sp, int eq, int reg, int pat);
  static const void *sweepv(int sp, int eq, int reg, int pat);
  static const void *sweepl(int sp, int eq, int reg, int tw);
  static const void *sweep_aa_shift(int sp, int eq, int reg);
  static const void *sweep_mfma(int sp, int reg);
  static const void *sweep_literal(int sp, int form);
  static const void *sweep_literal_cross(int form);
  static const void *sweep_force(int sp, int pat);
  static const void *sweep_cross(int pat);
  static const void *sweep_force_cross(int pat);
  static const void *init(int sp, int eq, int gm);
  static const void *exporter(int gm);
  static const void *importer(int gm);
  static const void *macro(int gm);
  static const void *diag(int gm);
};

const void *sweep_fn(int s, int store, int sp, int eq, int reg, int pat);
const void *sweepv_fn(int s, int store, int sp, int eq, int reg, int pat);
const void *sweepl_fn(int s, int store, int sp, int eq, int reg, int tw);
int sweepl_lds_bytes(int s, int store, int tw);
const void *sweep_aa_shift_fn(int s, int store, int sp, int eq, int reg);
const void *sweep_mfma_fn(int s, int store, int sp, int reg);
const void *sweep_literal_fn(int s, int store, int sp, int form);
const void *sweep_literal_cross_fn(int s, int store, int form);
const void *sweep_force_fn(int s, int store, int sp, int pat);
const void *sweep_cross_fn(int s, int store, int pat);
const void *sweep_force_cross_fn(int s, int store, int pat);
const void *init_fn(int s, int store, int sp, int eq, int gm);
const void *export_fn(int s, int store, int gm);
const void *import_fn(int s, int store, int gm);
const void *macro_fn(int s, int store, int gm);
const void *diag_fn(int s, int store, int gm);
const void *diag_final_fn();
const void *copy_fn();

}  // namespace lbm
