"""Build the CPU SIMT emulator binary: the library's kernel and C-ABI sources
compiled for the host against tests/simt/include/hip/hip_runtime.h, the CPU
oracle, and the emulator driver.  Test infrastructure only."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1105_6040_amd", "csrc")


def build(out_dir: str, sanitize: bool = True, opt: str = "-O1") -> str:
    os.makedirs(out_dir, exist_ok=True)
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"] if sanitize else []
    inc = [f"-I{os.path.join(HERE, 'include')}", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
    # -U_FORTIFY_SOURCE: the emulator longjmps between fiber stacks on purpose
    cxx = ["g++", "-std=c++17", opt, "-g", "-w", "-U_FORTIFY_SOURCE", *san, *inc]
    jobs = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp")):
            jobs.append((cxx + ["-x", "c++", "-c", os.path.join(CSRC, name)], name))
    jobs.append((cxx + ["-c", os.path.join(HERE, "simt.cpp")], "simt.cpp"))
    jobs.append((cxx + ["-c", os.path.join(HERE, "emu_driver.cpp")], "emu_driver.cpp"))
    jobs.append((["gcc", "-std=c11", opt, "-g", "-w", *san, "-c", os.path.join(ROOT, "oracle", "oracle.c")],
                 "oracle.c"))

    def run(job):
        cmd, name = job
        obj = os.path.join(out_dir, name + ".o")
        r = subprocess.run(cmd + ["-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile {name} failed:\n{r.stderr[-4000:]}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(run, jobs))
    exe = os.path.join(out_dir, "emu_driver")
    r = subprocess.run(["g++", *san, *objs, "-o", exe, "-lpthread"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    return exe


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(ROOT, "_work", "simt_build")))
