"""Build the gfx950 shared library libturpy.so in-tree with hipcc.

    python -m paper_2604_07248_amd.build
"""

import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libturpy.so")
POISON_LIB = os.path.join(HERE, "libturpy_poison.so")
SOURCES = ["kernels.hip", "receiver.hip", "api.hip", "host.cpp", "planner.cpp", "group.cpp", "batch.cpp"]

FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: plain FP32 VALU only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libturpy.so")
    return exe


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stderr[-8000:])
    return res.stderr


def build(verbose=False, poison=False, jobs=None):
    """Compile libturpy.so (always recompiles; one hipcc per source, in
    parallel, then one link); returns its path.  With poison=True, compile
    the test build libturpy_poison.so instead, whose kernels fill their LDS
    with NaN before using it (TURPY_LDS_POISON)."""
    out = POISON_LIB if poison else LIB
    extra = ["-DTURPY_LDS_POISON"] if poison else []
    with tempfile.TemporaryDirectory(prefix="turpy_build.") as d:
        def compile_one(src):
            obj = os.path.join(d, src + ".o")
            log = _run([hipcc()] + FLAGS + extra + ["-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src),
                                                   "-o", obj])
            return obj, log
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs or min(len(SOURCES), os.cpu_count() or 1)) as ex:
            done = list(ex.map(compile_one, SOURCES))
        fd, tmp = tempfile.mkstemp(prefix=os.path.basename(out)[:-len(".so")] + ".", suffix=".so.tmp", dir=HERE)
        os.close(fd)
        try:
            _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for o, _ in done] + ["-o", tmp])
        except RuntimeError:
            os.unlink(tmp)
            raise
    if verbose:
        sys.stderr.write("".join(log for _, log in done))
    os.replace(tmp, out)
    return out


def build_all(verbose=False):
    """The product library and its LDS-poison test build, side by side."""
    half = max(1, (os.cpu_count() or 2) // 2)
    with concurrent.futures.ThreadPoolExecutor(max_workers=2) as ex:
        jobs = [ex.submit(build, verbose, p, half) for p in (False, True)]
        return [j.result() for j in jobs]


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
