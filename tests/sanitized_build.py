"""Builds the server driver (`tests/serve_driver.cpp`) against the library with
its host runtime under AddressSanitizer and UndefinedBehaviorSanitizer:
`tests/bin/serve_asan`.  (A ThreadSanitizer build of the same program finds
no GPU: under it the HIP runtime reports that no ROCm-capable device is
present, so none is built.)

Test infrastructure.  The translation units that hold no kernel (the server,
the launch sets, the entry points, error and timing state) are compiled again
with the sanitizer on their host code only; the kernel files are linked from
the library's own objects in `_build/` (built first by
`paper_2001_05291_amd.build`), so their device code is the library's.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from paper_2001_05291_amd import build as lib  # noqa: E402

BIN = os.path.join(HERE, "bin")
DRIVER = os.path.join(HERE, "serve_driver.cpp")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
ROCM_LIB = "/opt/rocm/lib"
# no kernel in these: all host code, compiled again with the sanitizer
HOST_SOURCES = ["common.cpp", "timing.cpp", "launchset.hip", "tabu.hip", "noalloc.hip",
                "fleet.cpp", "batch.cpp", "serve.cpp"]
VARIANTS = {
    "asan": "address,undefined",
}


def _host_flags(kind: str) -> list:
    return ["-Xarch_host", "-fsanitize=" + VARIANTS[kind], "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-g"]


def _compile(kind: str, src: str, verbose: bool) -> str:
    out_dir = os.path.join(lib.BUILD, kind)
    obj = os.path.join(out_dir, os.path.splitext(os.path.basename(src))[0] + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [lib.HIPCC, *lib.COMMON, *_host_flags(kind), *lang, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> list:
    """Needs the library's objects in `_build/` (paper_2001_05291_amd.build)."""
    os.makedirs(BIN, exist_ok=True)
    kernel_objs = [os.path.join(lib.BUILD, os.path.splitext(s)[0] + ".o")
                   for s in lib.SOURCES if s not in HOST_SOURCES]
    for o in kernel_objs:
        if not os.path.exists(o):
            raise FileNotFoundError(f"{o}: build the library first")
    jobs = []
    for kind in VARIANTS:
        os.makedirs(os.path.join(lib.BUILD, kind), exist_ok=True)
        jobs += [(kind, os.path.join(lib.CSRC, s)) for s in HOST_SOURCES] + [(kind, DRIVER)]
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda j: (j[0], _compile(j[0], j[1], verbose)), jobs))
    outs = []
    for kind, san in VARIANTS.items():
        exe = os.path.join(BIN, f"serve_{kind}")
        tmp = exe + ".tmp%d" % os.getpid()
        mine = [o for k, o in objs if k == kind]
        cmd = [CLANGXX, "-fsanitize=" + san, "-o", tmp, *mine, *kernel_objs,
               "-L" + ROCM_LIB, "-lamdhip64", "-Wl,-rpath," + ROCM_LIB, "-lpthread"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, exe)
        outs.append(exe)
    return outs


if __name__ == "__main__":
    print("\n".join(build(verbose="-q" not in sys.argv)))
