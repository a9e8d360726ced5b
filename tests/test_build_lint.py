"""The device code contains no scalar memory access with a misaligned
immediate offset (the scalar unit ignores the low bits of the base register,
so such an access would read the wrong dword) and no mixed-precision fma (an
fp16 conversion folded into the fma before it rounds differently at fp16
ties).  CPU only: compiles to gfx950 assembly and inspects it."""
import subprocess

from paper_2605_17869_amd import build


def test_lint_flags_a_misaligned_immediate():
    asm = "_Zk:\n\ts_load_dword s3, s[20:21], 0xff\n\ts_load_dwordx2 s[4:5], s[0:1], 0x10\n"
    assert build.smem_misaligned(asm) == [("_Zk", "s_load_dword s3, s[20:21], 0xff")]


def test_lint_flags_a_mixed_precision_fma():
    asm = "_Zk:\n\tv_fma_mixlo_f16 v1, s88, v3, v11\n\tv_fmac_f32_e32 v1, s4, v2\n"
    assert build.mixed_f16_fma(asm) == [("_Zk", "v_fma_mixlo_f16 v1, s88, v3, v11")]


def test_kernels_have_no_misaligned_scalar_offsets(tmp_path):
    jobs = []
    for src in sorted(build.CSRC.glob("*.hip")):
        out = tmp_path / (src.name + ".s")
        jobs.append((out, subprocess.Popen(build.device_asm_cmd(src, out))))
    for out, pr in jobs:
        assert pr.wait() == 0
        text = out.read_text()
        if "__global__" in (build.CSRC / out.name[:-2]).read_text():
            assert "s_load" in text     # the files with kernels do load arguments
        assert build.smem_misaligned(text) == []
        assert build.mixed_f16_fma(text) == []
