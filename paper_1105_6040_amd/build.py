"""Build the gfx950 shared library ``libmi355sort.so`` in-tree with hipcc.

Every HIP source under ``csrc/`` and the C-ABI layer are compiled for gfx950
only and linked into one shared object next to this file.  Run as a script or
call ``build()``; it always recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(HERE, "_build")
LIB_NAME = "libmi355sort.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, name))
    return out


RESOURCE_REMARKS = "-Rpass-analysis=kernel-resource-usage"


# Kernels held to a register budget on purpose, with the spill each may
# have (bytes per lane): the one-launch segment queue for 32-bit keys without
# values runs two workgroups per CU at 128 registers with a small spill,
# faster than one workgroup per CU without it.
BOUNDED_SPILLS = {"segqueue_kernel_x2": 32}


def spilling_kernels(remarks: str):
    """(kernel, bytes per lane) for every kernel whose resource-usage remark
    reports private scratch: register spills, which these kernels must not
    have (a spilled tile kernel loses its occupancy and its speed), beyond
    the bounded spills listed above."""
    out, name = [], None
    for ln in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", ln)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", ln)
        if m and int(m.group(1)) > 0:
            b = int(m.group(1))
            if any(k in (name or "") and b <= lim for k, lim in BOUNDED_SPILLS.items()):
                continue
            out.append((name, b))
    return out


def _compile(src: str, extra) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    remarks = [RESOURCE_REMARKS] if src.endswith(".hip") else []
    cmd = [HIPCC, *COMMON, *extra, *lang, *remarks, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    spills = spilling_kernels(r.stderr)
    if spills:
        raise RuntimeError(f"{src}: kernels spill registers to scratch: {spills}")
    if r.stderr.strip():
        # warnings other than the host pass not knowing the packed-fp32 feature
        lines = [ln for ln in r.stderr.splitlines()
                 if "packed-fp32-ops" not in ln and "kernel-resource-usage" not in ln and ln.strip()]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(extra=(), jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, list(extra)), srcs))
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH} from {len(srcs)} sources")
    return LIB_PATH


def clean():
    shutil.rmtree(BUILD_DIR, ignore_errors=True)


if __name__ == "__main__":
    build()
