"""Build the HIP library libmlfft.so for gfx950, in-tree.

    python -m paper_2506_20350_amd.build [-j N] [-v] [--incremental]

Generates the FFT codelet header, compiles every source in csrc/ with hipcc
(--offload-arch=gfx950, packed-FP32 instructions disabled) in parallel and
links paper_2506_20350_amd/lib/libmlfft.so.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libmlfft.so")

SOURCES = ["fft2d.hip", "bgemm.hip", "bgemm_f32.hip", "bgemm_f64.hip", "bgemm_bf16.hip", "setup.hip", "krylov.hip", "net.hip", "lib.cpp", "solve.cpp", "netapi.cpp", "tune.cpp", "noalloc.hip", "dense.hip", "direct.cpp", "spectrum.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result", "-I", CSRC, "-I", os.path.join(ROOT, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)
    return out


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only sources newer than their object, or all of
    them when a header, the codelet generator or this script changed) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    hdr = os.path.join(CSRC, "fft_codelets.h")
    if not (incremental and os.path.exists(hdr) and os.path.getmtime(hdr) >= os.path.getmtime(os.path.join(CSRC, "gen_fft.py"))):
        _run([sys.executable, os.path.join(CSRC, "gen_fft.py"), hdr, "32"], verbose)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in srcs]
    jobs = jobs or min(8, os.cpu_count() or 1)

    def comp(i):
        return _run([HIPCC] + CFLAGS + ["-c", os.path.join(CSRC, srcs[i]), "-o", objs[i]], verbose)

    todo = list(range(len(srcs)))
    if incremental:
        deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
        deps += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
        deps.append(os.path.abspath(__file__))
        newest_dep = max(os.path.getmtime(d) for d in deps)
        todo = [i for i in todo if not os.path.exists(objs[i]) or
                os.path.getmtime(objs[i]) < max(newest_dep, os.path.getmtime(os.path.join(CSRC, srcs[i])))]
    # the heaviest translation units first
    order = sorted(todo, key=lambda i: -os.path.getsize(os.path.join(CSRC, srcs[i])))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(comp, order))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--incremental", action="store_true", help="recompile only what changed")
    a = ap.parse_args()
    print(build(a.j, a.v, a.incremental))


if __name__ == "__main__":
    main()
