"""Compile tests/host/exact_shim.cpp (the library's decision code, host build) with g++."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "_build", "libexact_shim.so")


def build():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    src = os.path.join(HERE, "exact_shim.cpp")
    deps = [src] + [os.path.join(HERE, "..", "..", "paper_1801_05745_amd", "csrc", f) for f in ("exact.hpp", "ring.hpp", "common.hpp")]
    if os.path.exists(OUT) and all(os.path.getmtime(OUT) >= os.path.getmtime(d) for d in deps):
        return OUT
    tmp = f"{OUT}.{os.getpid()}.tmp"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                    src, "-o", tmp], check=True)
    os.replace(tmp, OUT)
    return OUT
