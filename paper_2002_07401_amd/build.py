"""Compile the gfx950 HIP library libqmc_jagp.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqmc_jagp.so")
SOURCES = ["qmc_abi.hip", "gemm.hip", "linalg.hip", "eval.hip", "move.hip", "sweep.hip", "adjoint.hip", "multi.hip",
           "lrdmc.hip", "jas3.hip", "estimators.hip", "pfaff.hip", "ozaki.hip"]
ARCH = os.environ.get("QMC_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]
# per-source additions: the persistent sweep's move loop is compiled without
# machine loop-invariant code motion (see sweep.hip)
EXTRA = {"sweep.hip": ["-mllvm", "-disable-machine-licm"]}
NOISE = "is not a recognized feature for this target"


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if NOISE not in l)
    return res.returncode, err


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link libqmc_jagp.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="qmc_build_") as td:
        cmds = [[hipcc, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src),
                 "-o", os.path.join(td, src.replace(".hip", ".o"))] for src in SOURCES]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            results = list(ex.map(_run, cmds))
        for src, (rc, err) in zip(SOURCES, results):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src} ({rc}):\n{err}")
            if verbose and err.strip():
                print(err, file=sys.stderr)
        link = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}",
                *[os.path.join(td, s.replace(".hip", ".o")) for s in SOURCES], "-o", tmp]
        rc, err = _run(link)
        if rc != 0:
            raise RuntimeError(f"link failed ({rc}):\n{err}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
