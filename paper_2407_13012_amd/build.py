"""Build the gfx950 shared library libqaoa.so in-tree with hipcc.

Each source is compiled to an object in parallel, then the objects are linked
into the shared library (no device code crosses translation units)."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libqaoa.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "batch.hip", "mpnn.hip", "api.cpp", "plan.cpp", "lbfgs.cpp", "cost_terms.cpp", "noalloc.hip")]
# passes.hip is compiled once per precision and spectator class (see its header)
PASS_SOURCE = os.path.join(HERE, "csrc", "passes.hip")
PASS_VARIANTS = [(real, sp) for real in ("double", "float") for sp in (-1, 0, 2, 3, 4, 5, 6, 7)]


def units() -> list[tuple[str, list[str], str]]:
    """(source, extra flags, object name) of every translation unit."""
    out = [(s, [], os.path.basename(s) + ".o") for s in SOURCES]
    for real, sp in PASS_VARIANTS:
        tag = f"{'c128' if real == 'double' else 'c64'}_{'rt' if sp < 0 else 's%d' % sp}"
        out.append((PASS_SOURCE, [f"-DQK_PASS_REAL={real}", f"-DQK_PASS_SP={sp}"], f"passes_{tag}.o"))
    return out
ARCH = os.environ.get("QAOA_OFFLOAD_ARCH", "gfx950")


def compile_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # packed fp32 instructions are disabled for every HIP translation unit
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-result",
        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
    ]


def build(verbose: bool = False, jobs: int = 0) -> str:
    jobs = jobs or min(len(units()), os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="qaoa_build_") as tmpd:
        us = units()
        objs = [os.path.join(tmpd, o) for _, _, o in us]
        cmds = [["hipcc", *compile_flags(), *fl, "-c", s, "-o", o] for (s, fl, _), o in zip(us, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)

        def run(c):
            return subprocess.run(c, capture_output=True, text=True)

        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(run, cmds))
        for c, r in zip(cmds, results):
            if verbose and r.stderr:
                print(r.stderr, end="", file=sys.stderr, flush=True)
            if r.returncode != 0:
                if not verbose:
                    print(r.stderr, end="", file=sys.stderr, flush=True)
                raise subprocess.CalledProcessError(r.returncode, c)
        tmp = LIB + ".tmp"
        link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
