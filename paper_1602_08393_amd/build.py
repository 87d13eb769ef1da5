"""Builds libwmh.so (HIP for gfx950) in place: ``python -m paper_1602_08393_amd.build``."""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwmh.so")
SOURCES = ["wmh_host.cpp", "wmh_server.cpp", "wmh_kernels.hip", "wmh_walk.hip", "wmh_collide.hip",
           "wmh_index.hip",
           "wmh_tune.cpp", "wmh_codec.hip", "wmh_codec_host.cpp",
           "wmh_quantize.hip", "wmh_scale.cpp", "wmh_lsh.hip", "wmh_lsh_host.cpp",
           "wmh_noalloc.hip"]
ARCH = "gfx950"
# Per-file options.  The shared-window walk's branches are all scalar; leaving such regions
# unstructured lets its early loop exits leave the loop directly, which keeps the waits for its
# prefetched stream windows exact.
EXTRA = {"wmh_walk.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions"]}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
            "-Wno-unused-result", "-Wno-unused-value", "-munsafe-fp-atomics",
            # packed fp32 instructions stay off in every HIP object of this library
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]


# hipcc forwards -Xclang options to both the device and the host pass of each file, and the
# host pass reports the device-only feature as unknown (and ignores it).  That one notice is
# dropped from the build output; every other line of the compiler's output is shown.
_HOST_FEATURE_NOTICE = "'-packed-fp32-ops' is not a recognized feature for this target"


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, capture_output=True, text=True)
    for stream, text in ((sys.stdout, r.stdout), (sys.stderr, r.stderr)):
        lines = [ln for ln in text.splitlines() if _HOST_FEATURE_NOTICE not in ln]
        if lines:
            print("\n".join(lines), file=stream, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)


def build(verbose: bool = False) -> str:
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objects = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"]
        cmds.append([cc, *lang, *flags(), *EXTRA.get(src, []), "-c", os.path.join(CSRC, src),
                     "-o", obj])
        objects.append(obj)
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    # the files compile independently: a few at a time
    workers = max(1, min(len(cmds), (os.cpu_count() or 1), 8))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        for f in [pool.submit(_run, cmd) for cmd in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", *objects, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
