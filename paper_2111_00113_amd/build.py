"""Build the gfx950 HIP library libsgmres.so in-tree with hipcc.

Every translation unit under csrc/ is compiled to an object in parallel, then
linked into paper_2111_00113_amd/libsgmres.so.  Always rebuilds when called.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libsgmres.so")
OBJ_DIR = os.path.join(PKG, "_build")
ARCH = os.environ.get("SGMRES_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no floating-point contraction: fused multiply-adds are written out
    # (madd, gs_sub), so kernel instances that must agree bit for bit do the
    # same operations whatever the compiler schedules
    "-ffp-contract=off",
    f"-I{os.path.join(ROOT, 'include')}",
]

SOURCES = ["sell.hip", "arnoldi.hip", "arnoldi_sb.hip", "arnoldi_f32.hip", "arnoldi_bf16.hip", "arnoldi_halo_f64.hip", "arnoldi_halo_f32.hip", "arnoldi_halo_bf16.hip", "arnoldi_multi.hip", "batched.hip", "box.hip", "capi.hip", "chebyshev.hip", "lsq.hip", "multi.hip", "sketch.hip", "sketch_basis.hip", "stream.hip", "transpose.hip", "vec.hip"]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(ln for ln in res.stderr.splitlines() if noise not in ln)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
