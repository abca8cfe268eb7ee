"""Build the HIP library ``libmbw.so`` for gfx950 with hipcc (in-tree), and beside it the
measurement helper ``libmbw_probe.so`` (copy and random-gather probes used by the benchmark)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmbw.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["index_build.hip", "seed.hip", "serve.hip", "rescue.hip", "chain.hip", "debug.hip"]
PROBE_SRC = os.path.join(HERE, "probe", "probe.hip")
PROBE_OUT = os.path.join(HERE, "libmbw_probe.so")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
         # keep the compiler from forming packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "hipcc")

    def compile_one(src):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [hipcc, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if verbose:
            sys.stderr.write(r.stderr)
        return obj

    def build_probe():
        tmp = PROBE_OUT + ".tmp"
        r = subprocess.run([hipcc, *FLAGS, "-shared", "-o", tmp, PROBE_SRC], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for the probe library:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, PROBE_OUT)

    with ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        probe = ex.submit(build_probe)
        objs = list(ex.map(compile_one, SOURCES))
        probe.result()
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
