"""Build libmcv.so (HIP for gfx950 + the C ABI) in-tree with hipcc.

Every source is compiled for gfx950 only.  Packed FP32 instructions are kept
out of the generated code (-packed-fp32-ops target feature off).  The
adaptation kernels (adapt.hip) decide integers from floating-point values
(the largest-remainder allocation, the rebinning walk) and repeat the plain
IEEE sequence of their definition, so that translation unit is compiled with
floating-point contraction off (no fused multiply-adds the source does not
write).
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmcv.so")
SOURCES = ["single_f64.hip", "single_f32.hip", "mrg_f64.hip", "mrg_f32.hip", "trace_f64.hip",
           "trace_f32.hip", "sample.hip", "capi.hip", "jobs.hip", "batch.hip", "serve.hip",
           "adapt.hip", "noalloc.hip", "strat.hip"]
ARCH = "gfx950"
# per-source flags on top of common_flags()
EXTRA_FLAGS = {"adapt.hip": ["-ffp-contract=off"]}
# The batched sample kernel (queue.hip) is compiled once per precision, launch
# bound and term-bound option, so that its variants compile in parallel.
QUEUE_VARIANTS = [(prec, lb, tb) for prec in ("f32", "f64") for lb in (256, 512, 1024)
                  for tb in (1, 0)]


def units():
    """(object name, source, extra flags) of every object of the library."""
    out = [(f"queue_{p}_{lb}_{tb}.o", "queue.hip",
            [f"-DMCV_QUEUE_FP32={1 if p == 'f32' else 0}", f"-DMCV_QUEUE_LB={lb}",
             f"-DMCV_QUEUE_TB={tb}"]) for p, lb, tb in QUEUE_VARIANTS]
    # the slowest objects first, so that the pool never waits on one at the end
    out += [(src.replace(".hip", ".o"), src, EXTRA_FLAGS.get(src, [])) for src in SOURCES]
    return out


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
            "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _newest_input(src: str) -> float:
    """Latest modification time of a source, the headers and this script."""
    paths = [os.path.join(CSRC, src), os.path.abspath(__file__)]
    paths += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    paths += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    return max(os.path.getmtime(p) for p in paths)


def build(verbose: bool = False, jobs: int = 10, incremental: bool = False) -> str:
    """Compile every source (incremental: only those older than their inputs)
    and link libmcv.so."""
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(unit):
        name, src, extra = unit
        obj = os.path.join(objdir, name)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _newest_input(src):
            return obj
        cmd = [cc, "-c", os.path.join(CSRC, src), "-o", obj] + common_flags() + extra
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {name}:\n{r.stdout}")
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, units()))
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
