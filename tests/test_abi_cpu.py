"""C-ABI checks that need no GPU: the library loads, exports every symbol declared in
include/lbm.h, and validates parameters in pure host code (sec. 3 restrictions)."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2211_02435_amd import lbm
import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lbm.load()
    names = _declared_functions()
    assert len(names) >= 30
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)
    assert set(names) == set(lbm.SIGNATURES), set(names) ^ set(lbm.SIGNATURES)


def test_version_and_defaults():
    lib = lbm.load()
    assert b"gfx950" in lib.lbm_version()
    p = lbm.LbmParams()
    assert lib.lbm_params_default(p) == 0
    assert p.stencil == 2 and p.space == 2 and p.zero_centered == 1 and p.storage == 1
    assert list(p.periodic) == [1, 1, 1]


def _p(**kw):
    st = kw.pop("stencil", "D3Q27")
    om = kw.pop("omegas", O.regularized_rates(st, 1.9))
    dims = kw.pop("dims", (8, 8, 8) if st != "D2Q9" else (8, 8, 1))
    return lbm.make_params(st, kw.pop("space", "cumulant"), om, dims, **kw)


def test_absolute_storage_accepted_for_the_maxwellian():
    assert lbm.lbm_validate(_p(space="raw", zero_centered=0)) == 0
    assert lbm.lbm_validate(_p(space="cumulant", zero_centered=0)) == 0
    assert lbm.lbm_validate(_p(space="raw", zero_centered=0, eq_form="delta")) == lbm.LBM_EUNSUPPORTED


def test_valid_parameter_sets():
    for st in ("D2Q9", "D3Q19", "D3Q27"):
        for sp in ("raw", "central", "cumulant"):
            assert lbm.lbm_validate(_p(stencil=st, space=sp)) == 0, lbm.last_error()
    assert lbm.lbm_validate(_p(stencil="D2Q9", space="central", equilibrium="swe", gravity=0.1)) == 0
    # planes are rounded up to 256 bytes (plus the default padding)
    b32 = lbm.lbm_required_bytes(_p(dims=(10, 6, 4), storage="f32"))
    assert b32 % (2 * 27 * 256) == 0 and b32 >= 2 * 27 * 256 * 4
    b16 = lbm.lbm_required_bytes(_p(dims=(10, 6, 4), storage="f16", streaming="aa"))
    assert lbm.lbm_required_bytes(_p(dims=(10, 6, 4), storage="f16", streaming="esoteric")) == b16
    assert lbm.lbm_required_bytes(_p(dims=(10, 6, 4), storage="f16", streaming="twist")) == b16
    assert b16 % (27 * 256) == 0 and b16 >= 27 * 240 * 2


@pytest.mark.parametrize("kw,code", [
    (dict(stencil="D3Q27", omegas=np.ones(26)), lbm.LBM_EINVAL),
    (dict(dims=(0, 4, 4)), lbm.LBM_EINVAL),
    (dict(omegas=np.r_[np.zeros(4), np.full(23, 2.5)]), lbm.LBM_EINVAL),
    (dict(omegas=np.r_[np.zeros(4), np.full(22, 1.0), [np.nan]]), lbm.LBM_EINVAL),
    (dict(stencil="D2Q9", space="central", equilibrium="swe", gravity=0.0), lbm.LBM_EINVAL),
    (dict(space="cumulant", eq_form="delta"), lbm.LBM_EUNSUPPORTED),
    (dict(space="raw", eq_form="delta", zero_centered=0), lbm.LBM_EUNSUPPORTED),
    (dict(stencil="D2Q9", space="central", equilibrium="swe", gravity=0.1, zero_centered=0), lbm.LBM_EUNSUPPORTED),
    (dict(stencil="D2Q9", dims=(8, 8, 2)), lbm.LBM_EUNSUPPORTED),
    (dict(stencil="D3Q27", space="central", equilibrium="swe", gravity=0.1), lbm.LBM_EUNSUPPORTED),
    (dict(stencil="D2Q9", space="cumulant", equilibrium="swe", gravity=0.1), lbm.LBM_EUNSUPPORTED),
    (dict(dims=(65536, 4096, 2), storage="f32", layout="rows"), lbm.LBM_EUNSUPPORTED),
    # 2^32 cells of D3Q19 in F16 with AA: 163 GB, small z-planes, but 32-bit cell indices
    (dict(stencil="D3Q19", space="raw", dims=(2048, 2048, 1024), storage="f16", streaming="aa",
          omegas=O.regularized_rates("D3Q19", 1.2)), lbm.LBM_EUNSUPPORTED),
    (dict(layout="diagonal"), None),
    (dict(space="srt", omegas=np.r_[np.zeros(4), np.full(22, 1.2), [1.3]]), lbm.LBM_EINVAL),
    (dict(stencil="D2Q9", space="srt", omegas=np.r_[np.zeros(3), np.full(6, 1.2)], equilibrium="swe",
          gravity=0.1), lbm.LBM_EUNSUPPORTED),
    (dict(stencil="D3Q19", space="raw", arithmetic="literal"), lbm.LBM_EUNSUPPORTED),
    (dict(space="raw", arithmetic="literal", streaming="aa"), lbm.LBM_EUNSUPPORTED),
    (dict(space="raw", arithmetic="literal", streaming="esoteric"), lbm.LBM_EUNSUPPORTED),
    (dict(space="raw", arithmetic="literal", streaming="twist"), lbm.LBM_EUNSUPPORTED),
    (dict(space="raw", arithmetic="literal", streaming="push"), lbm.LBM_EUNSUPPORTED),
    (dict(space="cumulant", arithmetic="literal", eq_form="delta"), lbm.LBM_EUNSUPPORTED),
])
def test_invalid_parameter_sets(kw, code):
    if code is None:  # an unknown layout name never reaches the library
        with pytest.raises(KeyError):
            _p(**kw)
        return
    assert lbm.lbm_validate(_p(**kw)) == code
    assert lbm.last_error() != ""


def test_layout_enum_checked_and_large_boxes_accepted():
    p = _p()
    p.layout = 7
    assert lbm.lbm_validate(p) == lbm.LBM_EINVAL
    p = _p()
    p.streaming = 5
    assert lbm.lbm_validate(p) == lbm.LBM_EINVAL
    # push keeps two buffers like pull
    assert lbm.lbm_required_bytes(_p(dims=(10, 6, 4), storage="f32", streaming="push")) == \
        lbm.lbm_required_bytes(_p(dims=(10, 6, 4), storage="f32", streaming="pull"))
    # one population plane beyond 4 GiB is fine: population bases are 64-bit scalars
    assert lbm.lbm_validate(_p(dims=(2048, 2048, 256), storage="f32", layout="planes")) == 0
    # the largest rows z-planes below 4 GiB (x padded to 256 bytes) pass; one more row is refused
    assert lbm.lbm_validate(_p(dims=(6250, 6340, 2), storage="f32", layout="rows")) == 0
    assert lbm.lbm_validate(_p(dims=(6250, 6341, 2), storage="f32", layout="rows")) == lbm.LBM_EUNSUPPORTED
    assert lbm.lbm_validate(_p(dims=(4420, 4470, 2), storage="f64", layout="rows")) == 0
    assert lbm.lbm_validate(_p(dims=(4420, 4471, 2), storage="f64", layout="rows")) == lbm.LBM_EUNSUPPORTED
    assert lbm.lbm_validate(_p(dims=(6250, 6341, 2), storage="f32", layout="auto")) == 0
    # a rows z-plane of 29 GiB is refused, but AUTO falls back to planes (1 GiB z-planes)
    assert lbm.lbm_validate(_p(dims=(65536, 4096, 2), storage="f32", layout="rows")) == lbm.LBM_EUNSUPPORTED
    assert lbm.lbm_validate(_p(dims=(65536, 4096, 2), storage="f32", layout="auto")) == 0
    assert lbm.lbm_required_bytes(_p(dims=(65536, 4096, 2), storage="f32", layout="auto")) == \
        lbm.lbm_required_bytes(_p(dims=(65536, 4096, 2), storage="f32", layout="planes"))


def test_srt_and_literal_parameter_sets():
    for st in ("D2Q9", "D3Q19", "D3Q27"):
        q = lbm.Q[st]
        om = np.r_[np.zeros(3 if st == "D2Q9" else 4), np.full(q - (3 if st == "D2Q9" else 4), 1.3)]
        assert lbm.lbm_validate(_p(stencil=st, space="srt", omegas=om)) == 0, lbm.last_error()
    for st in ("D2Q9", "D3Q27"):
        for sp in ("raw", "central", "cumulant", "srt"):
            om = O.regularized_rates(st, 1.0) if sp == "srt" else O.regularized_rates(st, 1.7)
            for zc, form in ((0, "default"), (1, "absolute"), (1, "delta"), (1, "default")):
                if sp == "cumulant" and form == "delta":
                    continue
                for store in ("f64", "f32", "f16"):
                    p = _p(stencil=st, space=sp, omegas=om, zero_centered=zc, eq_form=form, storage=store,
                           arithmetic="literal")
                    assert lbm.lbm_validate(p) == 0, (st, sp, zc, form, store, lbm.last_error())
    p = _p()
    p.arithmetic = 2
    assert lbm.lbm_validate(p) == lbm.LBM_EINVAL
    p = _p(force=(1e-4, 0, 0), force_model="he")
    assert lbm.lbm_validate(p) == 0
    p.force_model = 2
    assert lbm.lbm_validate(p) == lbm.LBM_EINVAL


def test_d3q15_parameter_sets():
    """D3Q15 runs in every space with the Maxwellian equilibrium, on every storage and
    streaming pattern; the shallow-water equilibria, the literal arithmetic and the
    weighted-orthogonal basis are rejected."""
    om = O.regularized_rates("D3Q15", 1.6)
    srt = np.r_[np.zeros(4), np.full(11, 1.6)]
    for store in ("f64", "f32", "f16"):
        for stream in ("pull", "push", "aa", "esoteric", "twist"):
            for sp, w in (("raw", om), ("srt", srt), ("central", om), ("cumulant", om)):
                p = _p(stencil="D3Q15", space=sp, omegas=w, storage=store, streaming=stream)
                assert lbm.lbm_validate(p) == 0, (sp, store, stream, lbm.last_error())
    assert lbm.lbm_validate(_p(stencil="D3Q15", space="raw", omegas=om, force=(1e-5, 0, 0))) == 0
    assert lbm.lbm_validate(_p(stencil="D3Q15", space="raw", omegas=om, zero_centered=0)) == 0
    for kw in (dict(space="raw", arithmetic="literal"),
               dict(space="raw", equilibrium="swe", gravity=0.1)):
        assert lbm.lbm_validate(_p(stencil="D3Q15", omegas=om, **kw)) == lbm.LBM_EUNSUPPORTED, kw
        assert lbm.last_error() != ""
    assert lbm.lbm_validate(_p(stencil="D3Q15", space="raw", omegas=np.ones(27))) == lbm.LBM_EINVAL
    assert lbm.lbm_required_bytes(_p(stencil="D3Q15", space="raw", omegas=om, dims=(10, 6, 4),
                                     storage="f32")) % (2 * 15 * 256) == 0


def test_weighted_orthogonal_basis_parameter_sets():
    """The orthogonal bases (WO, O) are accepted for raw-moment MRT on D2Q9, D3Q19 and D3Q27
    (any storage and streaming pattern) and rejected elsewhere."""
    for st in ("D2Q9", "D3Q19", "D3Q27"):
        om = O.regularized_rates(st, 1.6)
        for store in ("f64", "f32", "f16"):
            for stream in ("pull", "push", "aa", "esoteric", "twist"):
                for basis in ("weighted_orthogonal", "orthogonal"):
                    p = _p(stencil=st, space="raw", omegas=om, storage=store, streaming=stream, basis=basis)
                    assert lbm.lbm_validate(p) == 0, (st, store, stream, basis, lbm.last_error())
    om = O.regularized_rates("D3Q27", 1.6)
    for kw in (dict(space="central"), dict(space="cumulant"), dict(space="srt", omegas=np.r_[np.zeros(4), np.full(23, 1.6)]),
               dict(stencil="D3Q15", space="raw", omegas=O.regularized_rates("D3Q15", 1.6)),
               dict(stencil="D2Q9", space="raw", omegas=O.regularized_rates("D2Q9", 1.6), equilibrium="swe",
                    gravity=0.1)):
        kw.setdefault("omegas", om)
        assert lbm.lbm_validate(_p(basis="weighted_orthogonal", **kw)) == lbm.LBM_EUNSUPPORTED, kw
        assert lbm.last_error() != ""
        assert lbm.lbm_validate(_p(basis="orthogonal", **kw)) == lbm.LBM_EUNSUPPORTED, kw
    for basis in ("weighted_orthogonal", "orthogonal"):
        assert lbm.lbm_validate(_p(space="raw", omegas=om, basis=basis, force=(1e-5, 0, 0), force_model="he")) == 0
        assert lbm.lbm_validate(_p(space="raw", omegas=om, basis=basis, arithmetic="literal", zero_centered=0)) == 0
    p = _p(space="raw", omegas=om)
    p.basis = 3
    assert lbm.lbm_validate(p) == lbm.LBM_EINVAL


def test_params_struct_layout_matches_the_header(tmp_path):
    """The ctypes mirror of lbm_params has the C compiler's size and field offsets."""
    fields = [f[0] for f in lbm.LbmParams._fields_]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "lbm.h"', "int main(void) {",
             '  printf("sizeof %zu\\n", sizeof(lbm_params));']
    lines += ['  printf("%s %%zu\\n", offsetof(lbm_params, %s));' % (f, f) for f in fields]
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    import ctypes
    assert int(out["sizeof"]) == ctypes.sizeof(lbm.LbmParams)
    for f in fields:
        assert int(out[f]) == getattr(lbm.LbmParams, f).offset, f


def test_nonperiodic_rejected():
    p = _p()
    p.periodic[2] = 0
    assert lbm.lbm_validate(p) == lbm.LBM_EUNSUPPORTED


def test_null_handles_are_rejected_without_a_device():
    """Every context and batch entry point checks its handle before touching a device."""
    import ctypes
    lib = lbm.load()
    EINVAL = -1
    out = (ctypes.c_double * 6)()
    assert lib.lbm_diagnostics_noalloc(None, out) == EINVAL
    assert lib.lbm_diagnostics(None, out) == EINVAL
    assert lib.lbm_set_staged(None, 1) == EINVAL
    assert lib.lbm_get_staged(None) == 0
    assert lib.lbm_set_vectorized(None, 1) == EINVAL
    assert lib.lbm_step(None, 3) == EINVAL
    assert lib.lbm_graph_prepare(None, 3) == EINVAL
    assert lib.lbm_autotune(None) == EINVAL
    ms = ctypes.c_double()
    assert lib.lbm_time_steps(None, 2, ctypes.byref(ms)) == EINVAL
    assert lib.lbm_batch_set_persistent(None, 1) == EINVAL
    assert lib.lbm_batch_get_persistent(None) == 0
    assert lib.lbm_batch_step(None, 2) == EINVAL
    assert lib.lbm_batch_autotune(None) == EINVAL
    assert lib.lbm_batch_time_steps(None, 2, ctypes.byref(ms)) == EINVAL
    assert lib.lbm_copy_bandwidth(None, None, 16, 1, None, ctypes.byref(ms)) == EINVAL
    assert lbm.last_error()


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No fallback: with the shared library absent every call raises instead of computing."""
    monkeypatch.setattr(lbm, "_lib", None)
    monkeypatch.setattr(lbm, "LIB_PATH", str(tmp_path / "libpaper_lbm.so"))
    with pytest.raises(RuntimeError, match="not found"):
        lbm.load()
    with pytest.raises(RuntimeError, match="not found"):
        lbm.Lattice("D3Q27", "cumulant", O.regularized_rates("D3Q27", 1.9), (8, 8, 8))


def test_plain_c_program_links_and_validates(tmp_path):
    """A C99 program includes lbm.h, links libpaper_lbm.so and runs the host-only calls
    (defaults, validation with its error text, required bytes) without a GPU."""
    src = tmp_path / "use.c"
    src.write_text(r'''
#include <stdio.h>
#include "lbm.h"
int main(void) {
  lbm_params p;
  double om[27];
  size_t bytes = 0;
  int i;
  if (lbm_params_default(&p) != LBM_OK) return 1;
  for (i = 0; i < 27; ++i) om[i] = 1.0;
  om[4] = om[5] = om[6] = om[7] = om[8] = 1.9;
  p.omegas = om;
  p.n_omegas = 27;
  p.nx = 64; p.ny = 32; p.nz = 16;
  if (lbm_validate(&p) != LBM_OK) return 2;
  if (lbm_required_bytes(&p, &bytes) != LBM_OK) return 3;
  printf("bytes %zu\n", bytes);
  p.n_omegas = 19;
  if (lbm_validate(&p) != LBM_EINVAL) return 4;
  printf("error %s\n", lbm_last_error());
  return 0;
}
''')
    exe = tmp_path / "use"
    libdir = os.path.dirname(lbm.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe),
                    "-L", libdir, "-lpaper_lbm", "-Wl,-rpath," + libdir], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    lines = dict(l.split(" ", 1) for l in r.stdout.splitlines())
    assert int(lines["bytes"]) == lbm.lbm_required_bytes(_p(dims=(64, 32, 16), storage="f32"))
    assert lines["error"] != ""
