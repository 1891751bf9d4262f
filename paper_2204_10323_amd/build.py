"""Build libflood.so for gfx950 in-tree with hipcc (and the benchmark's
bandwidth probe, bench_probe.so, beside bench.py)."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/flood_kernels.hip", "csrc/flood_fused.hip", "csrc/flood_adjoint.hip",
           "csrc/flood_runtime.hip"]
LIB = os.path.join(HERE, "libflood.so")
PROBE_SRC = os.path.join(ROOT, "bench_probe.hip")
PROBE_LIB = os.path.join(ROOT, "bench_probe.so")
OBJ_DIR = os.path.join(ROOT, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # No FMA contraction: a face computed by two work items must give the same bits.
    "-ffp-contract=off",
    # No packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _compile(src: str, obj: str, verbose: bool):
    cmd = [_hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _link(objs, out: str, verbose: bool):
    tmp = out + f".tmp{os.getpid()}"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile every translation unit (in parallel) and link libflood.so and
    bench_probe.so.  Always recompiles."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    units = [(os.path.join(HERE, s), os.path.join(OBJ_DIR, os.path.basename(s) + ".o"))
             for s in SOURCES]
    probe_obj = os.path.join(OBJ_DIR, "bench_probe.o")
    jobs = units + [(PROBE_SRC, probe_obj)]
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        for f in [ex.submit(_compile, s, o, verbose) for s, o in jobs]:
            f.result()
    _link([o for _, o in units], LIB, verbose)
    _link([probe_obj], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
