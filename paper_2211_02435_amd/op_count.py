"""Floating-point operation counts of the compiled collision kernels (sec. 4.3 and the
operation-count discussion that follows it).

The paper counts operations in the symbolic kernels its generator emits and states relative
findings: regularization removes a share of the operations that grows with the complexity of
the method (raw moments < central moments < cumulants), and the regularized cumulant kernel
costs 13 % (D3Q19) to 40 % (D3Q27) more operations than the SRT kernel.  This module counts
the same quantity in the gfx950 machine code of this library's sweep kernels, so those
relative findings can be set beside ours.

It compiles a kernel unit to device assembly with the library's own flags, splits the
assembly into functions, and counts the vector floating-point arithmetic instructions of
each pull-streaming sweep kernel: additions and subtractions, multiplications, fused
multiply-adds (two operations each), reciprocals and the division steps.  Loads, stores,
address and integer arithmetic are not counted, matching a count of the collision's
arithmetic.  The scalar sweep is straight-line per cell (one cell per lane), so the static
count is the per-cell count.  The graded-basis kernels are counted; the orthogonal-basis
variants (which add the cross-order blocks) are left out.

  python -m paper_2211_02435_amd.op_count [--storage f32|f64] [--json out.json]
"""
import argparse
import json
import os
import re
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

from . import build as B

STENCILS = {0: "D2Q9", 1: "D3Q19", 2: "D3Q27", 3: "D3Q15"}
SPACES = {0: "raw", 1: "central", 2: "cumulant", 3: "identity", 4: "srt"}
UNITS = {"D2Q9": "k_d2q9", "D3Q19": "k_d3q19", "D3Q27": "k_d3q27", "D3Q15": "k_d3q15"}

# mnemonic stem (without _e32/_e64/_dpp/_sdwa) -> (class, operations per instruction)
_OPS = {}
for t in ("f32", "f64"):
    for m in ("v_add_", "v_sub_", "v_subrev_"):
        _OPS[m + t] = ("add", 1)
    _OPS["v_mul_" + t] = ("mul", 1)
    for m in ("v_fma_", "v_fmac_", "v_fmaak_", "v_fmamk_", "v_mac_", "v_mad_"):
        _OPS[m + t] = ("fma", 2)
    _OPS["v_rcp_" + t] = ("rcp", 1)
    for m in ("v_div_scale_", "v_div_fmas_", "v_div_fixup_"):
        _OPS[m + t] = ("div", 1)
_SUFFIX = re.compile(r"_(e32|e64|dpp|sdwa)$")
_LABEL = re.compile(r"^(_Z\w+):")


def emit_assembly(unit, outdir):
    """Device assembly (.s) of one kernel unit, compiled with the library's flags."""
    src = os.path.join(B.CSRC, unit + ".hip")
    out = os.path.join(outdir, unit + ".s")
    cmd = [B.HIPCC] + B.HIP_FLAGS + ["--cuda-device-only", "-S", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("assembly failed: %s\n%s" % (" ".join(cmd), r.stderr[-2000:]))
    return out


def count_functions(path):
    """{mangled name: {class: instructions, 'ops': operations, 'branches': n}} per function."""
    funcs, cur = {}, None
    with open(path) as f:
        for line in f:
            m = _LABEL.match(line)
            if m:
                cur = funcs.setdefault(m.group(1), {"add": 0, "mul": 0, "fma": 0, "rcp": 0, "div": 0,
                                                    "ops": 0, "branches": 0})
                continue
            if cur is None:
                continue
            if line.startswith(".Lfunc_end"):
                cur = None
                continue
            s = line.strip()
            if not s or s[0] in ".;":
                continue
            mn = _SUFFIX.sub("", s.split()[0])
            if mn in _OPS:
                cls, n = _OPS[mn]
                cur[cls] += 1
                cur["ops"] += n
            elif mn.startswith("s_cbranch"):
                cur["branches"] += 1
    return funcs


def demangle(names):
    r = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True, text=True, check=True)
    return r.stdout.splitlines()


_SWEEP = re.compile(r"^void lbm::sweep_kernel<(\d+), (\d+), (\d+), (true|false), (\w+), (\w+), (\d+), (true|false)"
                    r"(?:, (true|false))?>")


def sweep_counts(storage="f32", stencils=("D3Q19", "D3Q27"), workdir=None):
    """Counts of the pull-streaming, unforced, Maxwellian sweep kernels of every space and
    both rate kinds; a list of dicts."""
    own = workdir is None
    workdir = workdir or tempfile.mkdtemp(prefix="lbm_asm_")
    units = [UNITS[s] + "_" + storage for s in stencils]
    with ThreadPoolExecutor(max_workers=len(units)) as ex:
        paths = list(ex.map(lambda u: emit_assembly(u, workdir), units))
    rows = []
    for path in paths:
        funcs = count_functions(path)
        names = list(funcs)
        for mangled, pretty in zip(names, demangle(names)):
            m = _SWEEP.match(pretty)
            if not m:
                continue
            s, sp, eq, reg, st, ct, pat, force, cross = m.groups()
            if eq != "0" or pat != "0" or force != "false" or int(sp) == 3 or cross == "true":
                continue
            c = funcs[mangled]
            rows.append(dict(stencil=STENCILS[int(s)], space=SPACES[int(sp)],
                             rates="regularized" if reg == "true" else "general", compute=ct, **c))
        if own:
            os.remove(path)
    if own:
        os.rmdir(workdir)
    order = {"srt": 0, "raw": 1, "central": 2, "cumulant": 3}
    rows.sort(key=lambda r: (r["stencil"], order[r["space"]], r["rates"] != "regularized"))
    return rows


def summary(rows):
    """The paper's relative measures on our counts: regularized cumulant over SRT, and the
    share of operations regularization removes per space."""
    by = {(r["stencil"], r["space"], r["rates"]): r["ops"] for r in rows}
    out = {}
    for st in sorted({r["stencil"] for r in rows}):
        srt = by.get((st, "srt", "regularized")) or by.get((st, "srt", "general"))
        k = by.get((st, "cumulant", "regularized"))
        if srt and k:
            out["%s R-K / SRT" % st] = k / srt
        for sp in ("raw", "central", "cumulant"):
            g, r = by.get((st, sp, "general")), by.get((st, sp, "regularized"))
            if g and r:
                out["%s %s saving by regularization" % (st, sp)] = 1.0 - r / g
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--storage", default="f32", choices=["f32", "f64"])
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    rows = sweep_counts(a.storage)
    print("%-6s %-9s %-12s %6s %6s %6s %6s %6s %8s %4s" % ("stencil", "space", "rates", "add", "mul", "fma",
                                                         "rcp", "div", "ops", "br"))
    for r in rows:
        print("%-6s %-9s %-12s %6d %6d %6d %6d %6d %8d %4d" % (r["stencil"], r["space"], r["rates"], r["add"],
                                                             r["mul"], r["fma"], r["rcp"], r["div"], r["ops"],
                                                             r["branches"]))
    s = summary(rows)
    for k, v in s.items():
        print("%-40s %.3f" % (k, v))
    if a.json:
        with open(a.json, "w") as f:
            json.dump({"storage": a.storage, "rows": rows, "summary": s}, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
