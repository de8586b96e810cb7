"""The C ABI used from a plain C99 program, without Python, PyTorch or ctypes: the program
creates a context whose buffers and stream the library allocates itself, initialises the
equilibrium from host arrays, steps, reads the populations back and destroys the context.
Its output is compared with the FP64 oracle (bar 1e-13 after 5 steps, as the parity tests).
"""
import os
import subprocess

import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
from paper_2211_02435_amd import lbm

pytestmark = pytest.mark.gpu

HEADER_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")

PROGRAM = r'''
#include <stdio.h>
#include <stdlib.h>
#include "lbm.h"

/* usage: prog <input> <output>; input: int64 stencil, space, storage, streaming, nx, ny, nz,
   steps, then q rates, ncells rho, 3 * ncells u (doubles); output: q * ncells doubles */
int main(int argc, char **argv) {
  long long h[8];
  FILE *f;
  lbm_params p;
  lbm_ctx *ctx = NULL;
  double *om, *rho, *u, *df;
  size_t nc, q;
  lbm_status s;
  if (argc != 3) return 64;
  f = fopen(argv[1], "rb");
  if (!f || fread(h, sizeof(long long), 8, f) != 8) return 65;
  q = h[0] == LBM_D2Q9 ? 9 : (h[0] == LBM_D3Q19 ? 19 : (h[0] == LBM_D3Q15 ? 15 : 27));
  nc = (size_t)h[4] * (size_t)h[5] * (size_t)h[6];
  om = malloc(q * sizeof(double));
  rho = malloc(nc * sizeof(double));
  u = malloc(3 * nc * sizeof(double));
  df = malloc(q * nc * sizeof(double));
  if (!om || !rho || !u || !df) return 66;
  if (fread(om, sizeof(double), q, f) != q || fread(rho, sizeof(double), nc, f) != nc ||
      fread(u, sizeof(double), 3 * nc, f) != 3 * nc)
    return 67;
  fclose(f);
  lbm_params_default(&p);
  p.stencil = (int)h[0];
  p.space = (int)h[1];
  p.storage = (int)h[2];
  p.streaming = (int)h[3];
  p.nx = h[4];
  p.ny = h[5];
  p.nz = h[6];
  p.omegas = om;
  p.n_omegas = (int)q;
  s = lbm_create(&p, &ctx);
  if (s == LBM_OK) s = lbm_init_equilibrium(ctx, rho, u);
  if (s == LBM_OK) s = lbm_step(ctx, h[7]);
  if (s == LBM_OK) s = lbm_get_populations(ctx, df);
  if (s != LBM_OK) {
    fprintf(stderr, "lbm error %d: %s\n", (int)s, lbm_last_error());
    if (ctx) lbm_destroy(ctx);
    return 1;
  }
  lbm_destroy(ctx);
  f = fopen(argv[2], "wb");
  if (!f || fwrite(df, sizeof(double), q * nc, f) != q * nc) return 68;
  fclose(f);
  printf("ok %zu cells\n", nc);
  return 0;
}
'''

CODES = {"stencil": {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2}, "space": {"raw": 0, "central": 1, "cumulant": 2},
         "storage": {"f64": 0}, "streaming": {"pull": 0, "aa": 1}}


@pytest.fixture(scope="module")
def program(tmp_path_factory):
    d = tmp_path_factory.mktemp("cprog")
    src = d / "run_lbm.c"
    src.write_text(PROGRAM)
    exe = d / "run_lbm"
    libdir = os.path.dirname(lbm.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-O1", "-Wall", "-Werror", "-I", HEADER_DIR, str(src), "-o", str(exe),
                    "-L", libdir, "-lpaper_lbm", "-Wl,-rpath," + libdir], check=True)
    return exe


@pytest.mark.parametrize("stencil,space,streaming,dims", [("D3Q27", "cumulant", "pull", (70, 9, 5)),
                                                          ("D3Q19", "raw", "aa", (70, 9, 5)),
                                                          ("D2Q9", "central", "pull", (70, 37, 1))])
def test_c_program_matches_oracle(program, tmp_path, stencil, space, streaming, dims):
    nx, ny, nz = dims
    steps = 5
    st = O.stencil(stencil)
    om = np.random.default_rng(4).uniform(0.8, 1.9, st.q)
    om[st.conserved] = 0.0
    rho, u = W.random_near_equilibrium_fields((nz, ny, nx), seed=6, drho=5e-3, umax=0.04)
    if st.d == 2:
        u[2] = 0.0
    head = np.array([CODES["stencil"][stencil], CODES["space"][space], CODES["storage"]["f64"],
                     CODES["streaming"][streaming], nx, ny, nz, steps], dtype=np.int64)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(head.tobytes())
        f.write(np.ascontiguousarray(om, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(rho, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(u, dtype=np.float64).tobytes())
    print("C program: %s %s %s %s, %d steps" % (stencil, space, streaming, dims, steps), flush=True)
    r = subprocess.run([str(program), str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    got = np.fromfile(out, dtype=np.float64).reshape(st.q, nz, ny, nx)
    m = O.Method(stencil, space, om)
    want = O.step(m, O.init_equilibrium(m, rho, u), steps)
    err = float(np.abs(got - want).max())
    print("C program %s %s %s: max|d df| = %.3e" % (stencil, space, streaming, err))
    assert err <= 1e-13
