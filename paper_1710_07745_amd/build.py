"""Build libcanny.so (all HIP sources, gfx950 only) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcanny.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # packed fp32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(HERE, "..", "include"),
]
# per-file extras: the strip walks unroll their row loops completely
# (sliding windows become register renaming), which needs a higher unroll
# limit; the differentiable kernels are split into radius groups so that
# those large compiles run in parallel
# the float kernels' inputs are finite by contract, so min/max need no NaN
# canonicalisation (-fno-honor-nans)
UNROLL = ["-mllvm", "-pragma-unroll-threshold=1000000"]
EXTRA = {
    "canny_f32_forward.hip": UNROLL + ["-fno-honor-nans"],
    "canny_u8_forward.hip": UNROLL,
    "canny_log.hip": UNROLL,
}
EXTRA.update({f"canny_mag_g{g}.hip": UNROLL + ["-fno-honor-nans"] for g in range(1, 7)})


def _headers_mtime() -> float:
    hdrs = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(HERE, "..", "include", "*.h"))
    return max((os.path.getmtime(h) for h in hdrs), default=0.0)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(os.path.getmtime(src), _headers_mtime()):
        return obj
    cmd = [HIPCC] + FLAGS + EXTRA.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every HIP source (incremental: only those older than their
    object file or any header) and link libcanny.so."""
    os.makedirs(OBJ, exist_ok=True)
    # the long (unrolled) compiles first, so they overlap the short ones
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")),
                  key=lambda f: (os.path.basename(f) not in EXTRA, f))
    jobs = jobs or min(8, os.cpu_count() or 4, len(srcs))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental), srcs))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "--incremental"]
    print(build(int(args[0]) if args else None, incremental="--incremental" in sys.argv))
