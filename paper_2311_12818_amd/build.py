"""Build libmpg.so (HIP, gfx950) in the package directory with hipcc.

Each translation unit is compiled to an object in parallel, then linked."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpg.so")
# the slowest units first, so that they start compiling at once
SOURCES = ["mpg_adjoint_plain_a.hip", "mpg_adjoint_plain_b.hip", "mpg_adjoint_plain_c.hip", "mpg_count_a.hip",
           "mpg_count_b.hip", "mpg_count_c.hip", "mpg_persistent.hip", "mpg_lib.hip", "mpg_trials.hip",
           "mpg_adjoint.hip", "mpg_guide.hip", "mpg_adjoint_plain.hip", "mpg_count.hip", "mpg_params.hip",
           "mpg_noalloc.hip", "mpg_stree.hip", "mpg_stree_build.hip", "mpg_train.cpp", "mpg_glossy.hip", "mpg_scene.cpp"]
HEADERS = ["mpg_device.h", "mpg_internal.h", "mpg_walk.h", "mpg_scene.h", "mpg_adjoint.h", "mpg_adjoint_plain.h",
           "mpg_count.h", "mpg_stree_build.h"]
DEPS = SOURCES + HEADERS

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # packed FP32 (v_pk_*_f32) stays off: only scalar FP32 VALU forms are emitted
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    # contraction into FMA only within one source expression: the same routine
    # rounds identically wherever it is inlined, so every form of the walk
    # (plain, persistent, lane refill) gives bit-identical results
    "-ffp-contract=on",
]


OBJDIR = os.path.join(HERE, "_build")


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every unit and links libmpg.so.  incremental=True keeps the
    objects in _build/ and recompiles only units older than their source or
    any header (a development convenience; the default builds from scratch)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(os.path.dirname(HERE), "include")]
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    headers = [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(os.path.dirname(HERE), "include", "mpg.h")]
    newest_header = max(os.path.getmtime(h) for h in headers if os.path.exists(h))
    with tempfile.TemporaryDirectory(prefix="mpg_build_") as tmpdir:
        objdir = OBJDIR if incremental else tmpdir
        os.makedirs(objdir, exist_ok=True)
        objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]

        def compile_one(k):
            src = os.path.join(CSRC, SOURCES[k])
            if incremental and os.path.exists(objs[k]) and \
                    os.path.getmtime(objs[k]) > max(os.path.getmtime(src), newest_header):
                return
            lang = ["-x", "hip"] if src.endswith(".hip") else []
            cmd = [hipcc, *HIPCC_FLAGS, *inc, *lang, "-c", src, "-o", objs[k]]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)

        with ThreadPoolExecutor(jobs) as pool:
            list(pool.map(compile_one, range(len(SOURCES))))
        tmp = LIB + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.exists(os.path.join(CSRC, d)) and os.path.getmtime(os.path.join(CSRC, d)) > t for d in DEPS)


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
