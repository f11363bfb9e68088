"""The per-operator VALU costs that bench.py reports as the operators' own
arithmetic (OP_VALU) against the AMD assembly of the library's operator
functions: each operator's common-path expression, as the interpreter
computes it per case, is compiled alone for gfx950 from the library source
and its vector instructions are counted (minus those of a plain copy
kernel); the interpreter's wavefront range compare adds one for sin, cos,
exp and the square root.  Host-only: hipcc cross-compiles, no GPU runs."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# opcode -> (expression of a and b, range compare added by the interpreter)
EXPR = {
    2: ("a + b", 0), 3: ("a - b", 0), 4: ("a * b", 0), 5: ("div_protected(a, b)", 0),
    6: ("sin_fast(a)", 1), 7: ("cos_fast(a)", 1), 8: ("exp_fast(a)", 1),
    9: ("log_protected(a)", 0), 10: ("__builtin_amdgcn_sqrtf(fabsf(a))", 1), 11: ("fabsf(a)", 0),
}


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    hipcc = _hipcc()
    if not hipcc:
        pytest.skip("no hipcc")
    sys.path.insert(0, ROOT)
    from paper_2607_06731_amd import _build
    d = tmp_path_factory.mktemp("opcost")
    src = os.path.join(ROOT, "paper_2607_06731_amd", "csrc", "gpeval.hip")
    lines = ['#include "%s"' % src,
             "__global__ void t_copy(float* __restrict__ x, const float* __restrict__ y)"
             " { const int i = threadIdx.x; x[i] = y[i]; }"]
    for op, (e, _) in EXPR.items():
        lines.append("__global__ void t_op%d(float* __restrict__ x, const float* __restrict__ y)"
                     " { const int i = threadIdx.x; const float a = x[i], b = y[i]; x[i] = %s; }"
                     % (op, e))
    probe = d / "probe.hip"
    probe.write_text("\n".join(lines) + "\n")
    flags = [f for f in _build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    out = d / "probe.s"
    subprocess.check_call([hipcc] + flags + ["--cuda-device-only", "-S", "-I",
                                             os.path.join(ROOT, "include"), "-o", str(out),
                                             str(probe)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return out.read_text()


def _valu(asm, name):
    m = re.search(r"^(_Z\d+%sPfPKf):[^\n]*\n(.*?)s_endpgm" % name, asm, re.S | re.M)
    assert m, name
    return sum(1 for l in m.group(2).splitlines() if re.match(r"\s+v_", l))


def test_op_valu_table_matches_the_assembly(asm):
    sys.path.insert(0, ROOT)
    import bench
    base = _valu(asm, "t_copy")
    for op, (_, rng) in EXPR.items():
        got = _valu(asm, "t_op%d" % op) - base + rng
        assert got == bench.OP_VALU[op], (op, got, bench.OP_VALU[op])
    assert bench.OP_VALU[0] == bench.OP_VALU[1] == 0
