"""Build libttcf.so (gfx950 kernels + C ABI runtime) in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libttcf.so")
SOURCES = [os.path.join(CSRC, "ttcf_kernels.hip"), os.path.join(CSRC, "ttcf_mlp.hip"),
           os.path.join(CSRC, "ttcf_capi.hip"), os.path.join(CSRC, "ttcf_channel.hip"),
           os.path.join(CSRC, "ttcf_channel_capi.hip"), os.path.join(CSRC, "ttcf_estimators.hip"),
           os.path.join(CSRC, "ttcf_elongation.hip")]
HEADERS = [os.path.join(CSRC, "ttcf_internal.h"), os.path.join(CSRC, "ttcf_channel.h"),
           os.path.join(os.path.dirname(HERE), "include", "ttcf.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 into paper_2312_02990_amd/libttcf.so."""
    if not force and not stale():
        return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose and res.stderr:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
