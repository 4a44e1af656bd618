"""Build the FP64 CPU oracle (test infrastructure) with gcc.

The oracle is compiled with -O2 -ffp-contract=off and without fast-math so that every
floating-point expression is evaluated exactly as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ttcf_oracle.c")
SOURCES = [SRC, os.path.join(HERE, "channel_oracle.c")]
LIB = os.path.join(HERE, "libttcf_oracle.so")


def build(force: bool = True) -> str:
    """Compile oracle/libttcf_oracle.so; returns its path."""
    if not force and os.path.exists(LIB) and all(
            os.path.getmtime(LIB) >= os.path.getmtime(x) for x in SOURCES):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-D_POSIX_C_SOURCE=200809L",
           "-o", tmp, *SOURCES, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
