"""Build liblbm.so for gfx950 in-tree with hipcc (one object per .hip source,
compiled in parallel, then linked)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["lbm_step.hip", "lbm_aux.hip", "lbm_adjoint.hip", "lbm_api.hip"]
# the fused-step kernels, one object per (storage form, collision model), so
# that the variants compile in parallel: (source, object, defines)
STORAGES = {"f32": "LBM_F32", "f16": "LBM_F16DEV", "bf16": "LBM_BF16DEV", "f64": "LBM_F64"}
COLLS = {"cm": 0, "cm1": 1, "bgk": 2, "rm": 3}
UNITS = [("lbm_step_inst.hip", f"lbm_step_{st}_{cn}.o", (f"LBM_STEP_ST={sv}", f"LBM_STEP_COLL={cv}"))
         for st, sv in STORAGES.items() for cn, cv in COLLS.items()]
UNITS += [(src, src.replace(".hip", ".o"), ()) for src in SOURCES]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _compile(src: str, build_dir: str = BUILD, defines=(), obj_name: str | None = None) -> str:
    obj = os.path.join(build_dir, obj_name or src.replace(".hip", ".o"))
    cmd = ["hipcc", *FLAGS, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile the sources (optionally with extra -D tuning switches) into `out`."""
    build_dir = BUILD if out == LIB else os.path.join(os.path.dirname(os.path.abspath(out)), "_build")
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(UNITS), max(1, os.cpu_count() or 1), 16)) as ex:
        objs = list(ex.map(lambda u: _compile(u[0], build_dir, (*defines, *u[2]), u[1]), UNITS))
    tmp = out + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
