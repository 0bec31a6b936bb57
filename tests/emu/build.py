"""Build the CPU emulation of the batched kernel (test infrastructure).

The emulator compiles the kernel's workgroup building blocks
(paper_2208_01239_amd/csrc/batched_dev.hpp) for the host with LLVM's clang++,
which understands the vector types the kernel code uses.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "batched_emu.cpp")
DEV = os.path.join(os.path.dirname(os.path.dirname(HERE)), "paper_2208_01239_amd", "csrc", "batched_dev.hpp")
OUT = os.path.join(HERE, "_build", "libbatched_emu.so")
CXX = os.environ.get("FROB_EMU_CXX", "/opt/rocm/llvm/bin/clang++")


def build(force: bool = False) -> str:
    fresh = os.path.exists(OUT) and os.path.getmtime(OUT) >= max(os.path.getmtime(SRC), os.path.getmtime(DEV))
    if fresh and not force:
        return OUT
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cmd = [CXX, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-Wno-psabi", "-o", OUT + ".tmp", SRC]
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(force=True))
