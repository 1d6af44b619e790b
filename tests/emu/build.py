"""Build the CPU emulation of the library (test infrastructure only).

The library's kernel and host sources are compiled with the host compiler
against hip/hip_runtime.h of this folder (each GPU thread a fiber, the lanes
of a wave meeting at every cross-lane operation; see emu_runtime.cpp) into
``_build/libxdrop_emu.so``, which exports the same C ABI as libxdrop.so.
Textual changes make the kernel source host C++: the GPU intrinsic
name bound to the write-lane declaration is dropped (the runtime defines the
function), the register-class letters of the empty optimisation-barrier asm
statements become the host's general class, the two bit-scan instructions
written as asm statements become calls of host functions of the runtime, and the occupancy hint on kernel
definitions (a register budget for the GPU compiler) is dropped; a trace
hook after the wave kernel's tier loop reports the tier each extension ends
on to the runtime, and every shared-memory declaration registers its
variable, which the runtime fills with garbage once per block (no code may
read LDS it has not written).  Nothing else differs.
The product never loads this library; only tests do.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2304_08662_amd", "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libxdrop_emu.so")
CXX = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")


def host_source(text: str) -> str:
    text = re.sub(r'__asm\(\s*"llvm\.amdgcn\.writelane\.i32"\s*\)', "", text)
    text = re.sub(r'"\+[sv]"', '"+r"', text)
    # the bit scans written as single instructions become host functions
    text = re.sub(r'asm\("v_ffb([lh])_(?:b32|u32) %0, %1" : "=v"\((\w+)\) : "v"\((\w+)\)\);',
                  r'\2 = emu_ffb\1_32(\3);', text)
    text = re.sub(r'__attribute__\(\(amdgpu_waves_per_eu\([^()]*\)\)\)', "", text)
    # shared variables start with garbage in every block
    def _shared(m):
        names = re.findall(r'(\w+)\s*(?:\[[^\]]*\])?\s*(?:,|$)', m.group(2))
        return m.group(0) + "".join(
            f" emu::shared_decl(&{n}, sizeof({n}));" for n in names)
    text = re.sub(r'^(\s*)__shared__\s+(?:[\w:<>, ]+?\s+)?((?:\w+\s*(?:\[[^\]]*\])?\s*,?\s*)+);',
                  _shared, text, flags=re.M)
    # trace hook: the tier each extension of the wave kernel ends on
    text = re.sub(r'(r = start_tier<ALPHA, CMIN, CMAX>\(e, w, tab, P, S, start, tier\);)',
                  r'\1 emu_item_done(item, r, tier);', text)
    return text


def build(csrc: str | None = None, out: str = LIB, extra=(),
          include: str | None = None) -> str:
    """Compile the emulation library.  csrc / include: another source tree
    of the library to build instead of this one (to examine older
    versions)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    csrc = csrc or CSRC
    ksrc = os.path.join(csrc, "xdrop_kernels.hip")
    with open(ksrc, encoding="utf-8") as f:
        k = host_source(f.read())
    # (per-process names: test workers may build at the same time)
    kout = f"{out}.{os.getpid()}.kernels.cpp"
    with open(kout, "w", encoding="utf-8") as f:
        f.write(k)
    srcs = [kout, os.path.join(csrc, "xdrop_host.cpp"),
            os.path.join(HERE, "emu_runtime.cpp")]
    if os.path.exists(os.path.join(csrc, "xdrop_server.cpp")):
        srcs.append(os.path.join(csrc, "xdrop_server.cpp"))
    cmd = [CXX, "-O2", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Wno-unused-command-line-argument", "-I", HERE, "-I",
           include or os.path.join(ROOT, "include"), "-I", csrc, *extra, *srcs, "-o", f"{out}.{os.getpid()}.tmp", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(f"{out}.{os.getpid()}.tmp", out)
    os.remove(kout)
    return out


if __name__ == "__main__":
    print(build())
