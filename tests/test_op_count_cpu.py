"""Host checks of the operation counter (paper_2211_02435_amd.op_count): instruction classes,
two operations per fused multiply-add, function boundaries, and the relative measures."""
from paper_2211_02435_amd import op_count as OC

ASM = """\t.text
_Z3fooPf:                              ; @_Z3fooPf
\tv_add_f32_e32 v0, v1, v2
\tv_sub_f32_e64 v0, v1, -v2
\tv_mul_f64 v[0:1], v[2:3], v[4:5]
\tv_fma_f32 v0, v1, v2, v3
\tv_fmac_f32_e32 v0, v1, v2
\tv_pk_add_f16 v0, v1, v2
\tv_rcp_f32_e32 v0, v1
\tv_div_scale_f32 v0, vcc, v1, v2, v1
\ts_cbranch_execz .LBB0_2
\tglobal_load_dword v0, v[0:1], off
\t; v_add_f32 in a comment
.Lfunc_end0:
\tv_add_f32_e32 v0, v1, v2
_Z3barv:
\tv_fmaak_f32 v0, v1, v2, 0x3e800000
.Lfunc_end1:
"""


def test_count_functions(tmp_path):
    p = tmp_path / "x.s"
    p.write_text(ASM)
    f = OC.count_functions(str(p))
    assert set(f) == {"_Z3fooPf", "_Z3barv"}
    foo = f["_Z3fooPf"]
    assert (foo["add"], foo["mul"], foo["fma"], foo["rcp"], foo["div"]) == (2, 1, 2, 1, 1)
    assert foo["ops"] == 2 + 1 + 4 + 1 + 1
    assert foo["branches"] == 1
    assert f["_Z3barv"]["fma"] == 1 and f["_Z3barv"]["ops"] == 2


def test_summary_ratios():
    rows = [dict(stencil="D3Q27", space="srt", rates="general", ops=500),
            dict(stencil="D3Q27", space="cumulant", rates="regularized", ops=700),
            dict(stencil="D3Q27", space="cumulant", rates="general", ops=1400)]
    s = OC.summary(rows)
    assert abs(s["D3Q27 R-K / SRT"] - 1.4) < 1e-12
    assert abs(s["D3Q27 cumulant saving by regularization"] - 0.5) < 1e-12


def test_demangle_matches_sweep_pattern():
    name = "_ZN3lbm12sweep_kernelILi2ELi2ELi0ELb1EffLi0ELb0ELb0EEEvNS_9SweepArgsIT3_T4_EE"
    pretty = OC.demangle([name])[0]
    m = OC._SWEEP.match(pretty)
    assert m and m.groups() == ("2", "2", "0", "true", "float", "float", "0", "false", "false")
