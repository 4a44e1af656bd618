"""Build libttcf.so (gfx950 kernels + C ABI runtime) in-tree with hipcc.

Each source compiles to its own object in parallel (_build/, git-ignored), then one link."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libttcf.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = [os.path.join(CSRC, f) for f in (
    "ttcf_kernels.hip", "ttcf_pairs.hip", "ttcf_mlp.hip", "ttcf_capi.hip", "ttcf_channel.hip",
    "ttcf_channel_capi.hip", "ttcf_estimators.hip", "ttcf_elongation.hip")]
HEADERS = [os.path.join(CSRC, "ttcf_internal.h"), os.path.join(CSRC, "ttcf_device.h"),
           os.path.join(CSRC, "ttcf_channel.h"),
           os.path.join(os.path.dirname(HERE), "include", "ttcf.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


def _compile(src: str) -> tuple:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    res = subprocess.run([HIPCC, *FLAGS, "-c", "-o", obj, src], capture_output=True, text=True)
    return src, obj, res


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 into paper_2312_02990_amd/libttcf.so."""
    if not force and not stale():
        return LIB
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        results = list(pool.map(_compile, SOURCES))
    errors = [f"{src}:\n{res.stdout}{res.stderr}" for src, _, res in results if res.returncode != 0]
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    if verbose:
        for src, _, res in results:
            if res.stderr:
                print(res.stderr)
    tmp = LIB + ".tmp"
    res = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp,
                          *[obj for _, obj, _ in results]], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
