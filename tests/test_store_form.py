"""CPU check of the gfx950 code this repository builds: every 128-bit buffer
store of the multi-order walks (propagation, recomputation, adjoint and
batched deep passes) carries its whole offset in the lane register with a
zero scalar offset.  With a register scalar offset the compiler omits the
wait state that the store's data registers need before the next VALU write,
and stored values were intermittently replaced by newer ones in some lanes;
this test keeps that form from coming back.  It reads the device code object
of the objects build() left in the package's _build folder (nothing is
generated or committed)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_0907_3022_amd", "_build")
LLVM = "/opt/rocm/llvm/bin"
STORE = re.compile(r"^\s*buffer_store_dwordx4\s+(\S+),\s*(\S+),\s*(\S+),\s*(\S+)")


def disassemble(obj, tmp_path):
    if not os.path.exists(obj):
        pytest.fail(f"{obj} is missing: run build() first")
    fat = str(tmp_path / (os.path.basename(obj) + ".fatbin"))
    co = str(tmp_path / (os.path.basename(obj) + ".co"))
    subprocess.check_call([f"{LLVM}/llvm-objcopy", "-O", "binary", "--only-section=.hip_fatbin", obj, fat])
    targets = subprocess.check_output([f"{LLVM}/clang-offload-bundler", "--list", "--type=o",
                                       f"--input={fat}"], text=True).split()
    tgt = [t for t in targets if t.endswith("gfx950")]
    assert tgt, targets
    subprocess.check_call([f"{LLVM}/clang-offload-bundler", "--type=o", f"--targets={tgt[0]}",
                           f"--input={fat}", f"--output={co}", "--unbundle"])
    return subprocess.check_output([f"{LLVM}/llvm-objdump", "-d", "--mcpu=gfx950", co], text=True)


def scalar_offsets(asm):
    """soffset operand of every 128-bit buffer store."""
    return [m.group(4) for m in map(STORE.match, asm.splitlines()) if m]


def test_parser_sees_register_scalar_offsets():
    asm = ("\tbuffer_store_dwordx4 v[6:9], v73, s[16:19], 0 offen nt\n"
           "\tbuffer_store_dwordx4 v[2:5], v7, s[8:11], s12 offen\n")
    assert scalar_offsets(asm) == ["0", "s12"]


@pytest.mark.parametrize("src", ["pair.hip", "adjoint.hip", "batch.hip"])
def test_deep_walk_stores_have_zero_scalar_offset(src, tmp_path):
    offs = scalar_offsets(disassemble(os.path.join(BUILD, src + ".o"), tmp_path))
    assert len(offs) > 100, "no 128-bit buffer stores found"
    bad = sorted(set(o for o in offs if o != "0"))
    assert not bad, f"128-bit buffer stores with scalar offsets {bad} in {src}"
