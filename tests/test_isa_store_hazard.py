"""Host-side checks of the compiled kernels (no GPU): no 12- or 16-byte
buffer store is followed at once by a vector-ALU write of its data
registers, and the two-particle step kernels keep their register budgets.

A buffer store of more than 8 bytes reads its data registers after it
issues, so a VALU write of them must wait one cycle.  The compiler inserts
that wait unless the store's scalar offset is a register; on gfx950 such a
store was seen to write the next instruction's results in some lanes.  The
kernels therefore give these stores a zero scalar offset, and this test
reads the gfx950 assembly of the sources that hold them to check that no
store is left unguarded."""

import functools
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1612_00746_amd", "csrc")
# one translation unit per kernel family with 16-byte stores
SOURCES = ["step3c.hip", "step2d_f64_p2_full.hip", "step2d_f32k_p2_vec.hip"]
STORE = re.compile(r"(buffer_store_dwordx[34]|buffer_store_format_xyzw?)\s+(v\[\d+:\d+\])")
VALU = re.compile(r"(v_\w+)\s+(v\[\d+:\d+\]|v\d+)")


def _hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def _regs(spec):
    m = re.match(r"v\[(\d+):(\d+)\]", spec)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", spec)
    return {int(m.group(1))} if m else set()


def unguarded_stores(asm: str):
    """(line, store, next instruction) for every >8-byte buffer store whose
    next instruction is a VALU write of one of its data registers."""
    lines = [l.strip() for l in asm.splitlines()]
    out = []
    for i, l in enumerate(lines):
        m = STORE.match(l)
        if not m:
            continue
        j = i + 1
        while j < len(lines) and (not lines[j] or lines[j][0] in ";."):
            j += 1
        nxt = lines[j] if j < len(lines) else ""
        v = VALU.match(nxt)
        if v and _regs(v.group(2)) & _regs(m.group(2)):
            out.append((i + 1, l, nxt))
    return out


def test_scanner_flags_an_unguarded_store():
    asm = """
    buffer_store_dwordx4 v[16:19], v121, s[8:11], s72 offen nt
    v_cndmask_b32_e32 v17, 0, v127, vcc
    buffer_store_dwordx4 v[20:23], v1, s[8:11], 0 offen nt
    s_nop 0
    v_mov_b32_e32 v20, 0
    buffer_store_dwordx2 v[30:31], v1, s[8:11], s5 offen
    v_mov_b32_e32 v30, 0
    """
    hits = unguarded_stores(asm)
    assert len(hits) == 1 and "v[16:19]" in hits[0][1]


_TMP = tempfile.mkdtemp(prefix="ctqw_isa_")


@functools.lru_cache(maxsize=None)
def _assembly(src: str) -> str:
    """gfx950 assembly of one translation unit (compiled once per session)."""
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not available")
    out = os.path.join(_TMP, src + ".s")
    cmd = [cc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "--cuda-device-only", "-S",
           os.path.join(CSRC, src), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    with open(out) as fh:
        return fh.read()


@pytest.mark.parametrize("src", SOURCES)
def test_no_store_data_overwritten_at_once(src):
    hits = unguarded_stores(_assembly(src))
    assert not hits, "\n".join(f"{n}: {a} / {b}" for n, a, b in hits[:5])


def kernel_resources(asm: str):
    """{(pipeline depth, kernel name): (VGPRs, scratch bytes per lane)} of
    the step kernels in an assembly listing."""
    out = {}
    for m in re.finditer(r"\.amdhsa_kernel (\S+)(.*?)\.end_amdhsa_kernel", asm, re.S):
        name, body = m.group(1), m.group(2)
        depth = re.search(r"step2d_kernelI[fd]Li(\d+)E", name)
        if not depth:
            continue
        vgpr = int(re.search(r"\.amdhsa_next_free_vgpr\s+(\d+)", body).group(1))
        scratch = int(re.search(r"\.amdhsa_private_segment_fixed_size\s+(\d+)", body).group(1))
        out[(int(depth.group(1)), name)] = (vgpr, scratch)
    return out


@pytest.mark.parametrize("src", ["step2d_f32k_p2_vec.hip", "step2d_f64_p2_full.hip"])
def test_step_kernels_keep_their_register_budget(src):
    """The sweep's occupancy rests on the kernels' register counts: the
    complex64 two-column kernels up to 7 terms fit 256 VGPRs (two waves per
    SIMD) and no step kernel spills.  Everything derived from the work
    item (its realisation, row bases, the claim of the next item) is
    wave-uniform and must stay in scalar registers: when the compiler
    loses track of that (a claim index it cannot prove uniform), the
    uniform values move to VGPRs, the order-7 complex64 kernel spills and
    the complex128 kernels drop to one wave per SIMD."""
    res = kernel_resources(_assembly(src))
    assert res, "no step kernels found"
    for (depth, name), (vgpr, scratch) in sorted(res.items()):
        assert scratch == 0, f"{name}: {scratch} bytes of scratch"
        if src.startswith("step2d_f32k") and depth <= 7:
            assert vgpr <= 256, f"{name}: {vgpr} VGPRs"
        if src.startswith("step2d_f64") and depth <= 3:
            assert vgpr <= 256, f"{name}: {vgpr} VGPRs"


def test_adjoint_passes_do_not_spill():
    """The K-level adjoint passes (forward vectors up to 8 / 4 levels,
    Horner passes up to 3 / 2 levels for complex64 / complex128) hold every
    level's rows in registers; none may spill to scratch."""
    asm = _assembly("adjoint_pipe.hip")
    found = 0
    for m in re.finditer(r"\.amdhsa_kernel (\S+)(.*?)\.end_amdhsa_kernel", asm, re.S):
        name, body = m.group(1), m.group(2)
        if "pipe_kernel" not in name:
            continue
        found += 1
        scratch = int(re.search(r"\.amdhsa_private_segment_fixed_size\s+(\d+)", body).group(1))
        vgpr = int(re.search(r"\.amdhsa_next_free_vgpr\s+(\d+)", body).group(1))
        assert scratch == 0 and vgpr <= 256, f"{name}: {vgpr} VGPRs, {scratch} bytes of scratch"
    # five layouts (one row, full grid and ring, triangle) x (8 + 3 complex64
    # and 4 + 2 complex128 depths)
    assert found == 5 * (8 + 3 + 4 + 2)

