"""Build libttsh.so for gfx950 with hipcc (cross-compiles without a GPU).

The kernels are compiled once per grid size (kernels_n.hip with -DTTSH_N=N)
in parallel, plus the host runtime, then linked into a shared library next to
this file.  Usage:  python -m paper_2304_03306_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent
CSRC = HERE / "csrc"
OUT = HERE / "_build"
LIB = HERE / "libttsh.so"
SIZES = (64, 128, 256, 512, 1024, 2048, 4096, 8192)
# the production sizes' step passes: (N, arithmetic) pairs whose tiles fit the LDS
BIG = ((4096, 32), (4096, 64), (4096, 96), (8192, 32), (8192, 96))
PRECS = (32, 64, 96)
BLOCKS = (64, 128, 256)
SCHED_VARIANTS = (6, 10, 9, 7, 11)  # kSchedVariants of csrc/launch.hpp
ARCH = os.environ.get("TTSH_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def sources():
    return sorted(CSRC.glob("*.hip")) + sorted(CSRC.glob("*.hpp")) + sorted((HERE.parent / "include").glob("*.h"))


def build(jobs: int | None = None, verbose: bool = True) -> Path:
    OUT.mkdir(exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    units = [(CSRC / "kernels_n.hip", OUT / f"kernels_{n}.o", [f"-DTTSH_N={n}"]) for n in SIZES]
    units += [(CSRC / "step_multi.hip", OUT / f"step_{p}_{b}.o", [f"-DTTSH_PREC={p}", f"-DTTSH_BS={b}"])
              for p in PRECS for b in BLOCKS]
    # the FP32 step passes with the other transform schedules the autotuner tries
    units += [(CSRC / "step_sched.hip", OUT / f"sched_{b}_{s}.o", [f"-DTTSH_BS={b}", f"-DTTSH_SCH={s}"])
              for b in BLOCKS for s in SCHED_VARIANTS]
    units += [(CSRC / "step_big.hip", OUT / f"big_{n}_{p}.o", [f"-DTTSH_N={n}", f"-DTTSH_PREC={p}"]) for n, p in BIG]
    units.append((CSRC / "ttsh_capi.hip", OUT / "ttsh_capi.o", []))
    units.append((CSRC / "fno.hip", OUT / "fno.o", []))
    units.append((CSRC / "stream.hip", OUT / "stream.o", []))
    cmds = [[HIPCC, *FLAGS, *extra, "-c", str(src), "-o", str(obj)] for src, obj, extra in units]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, fut in zip(cmds, [ex.submit(_run, c) for c in cmds]):
            fut.result()
            if verbose:
                print("compiled", cmd[-1], flush=True)
    tmp = LIB.with_suffix(".so.tmp")
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp),
          *[str(o) for _, o, _ in units]])
    os.replace(tmp, LIB)
    if verbose:
        print("linked", LIB, flush=True)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
