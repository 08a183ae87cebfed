"""Builds the HIP library paper_2009_05112_amd/libvegasp.so for gfx950 with hipcc.

Every translation unit is compiled with -ffp-contract=off (the arithmetic is
exactly what the source spells out; fused multiply-adds only where fma() is
written) and with packed FP32 instructions disabled.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvegasp.so")
EXAMPLES = os.path.join(HERE, "libvegasp_examples.so")  # example batched integrands
def _instances():
    import importlib.util
    spec = importlib.util.spec_from_file_location("gen_instances", os.path.join(CSRC, "gen_instances.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.sources()


# largest translation units first, so that they start compiling first
SOURCES = _instances() + ["vp_runtime.hip", "vp_server.hip", "vp_aux.hip"]
ARCH = os.environ.get("VEGASP_ARCH", "gfx950")
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def _compile(src):
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    extra = ["-Rpass-analysis=kernel-resource-usage"] if os.environ.get("VEGASP_RESOURCE_USAGE") else []
    cmd = [_hipcc()] + FLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msg}")
    return out, msg


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = min(len(SOURCES), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    for _, msg in results:
        if verbose and msg.strip():
            print(msg)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    # ROCTx ranges of the host-side phases (rocprofiler-sdk's marker library)
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    r = subprocess.run([_hipcc()] + FLAGS + ["-shared", os.path.join(CSRC, "vp_examples.hip"), "-o", EXAMPLES],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("vp_examples failed:\n" + r.stdout + r.stderr)
    if verbose:
        print("built", LIB, "and", EXAMPLES)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
