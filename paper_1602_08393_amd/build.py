"""Builds libwmh.so (HIP for gfx950) in place: ``python -m paper_1602_08393_amd.build``."""
from __future__ import annotations

import concurrent.futures
import hashlib
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
            f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]


# Device-only options: packed fp32 instructions stay off in every HIP object of this library.
# They are a feature of the GPU target, so they go to the device pass alone.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, capture_output=True, text=True)
    for stream, text in ((sys.stdout, r.stdout), (sys.stderr, r.stderr)):
        if text.strip():
            print(text.rstrip(), file=stream, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)


def _compile_cmds(cc: str, src: str, obj: str) -> list[list[str]]:
    """Two passes per file: the device code (with DEVICE_FLAGS) into a code-object bundle, then
    the host code with that bundle embedded.  Both passes share one compilation-unit id, which
    names the file's device symbols on both sides."""
    base = os.path.splitext(obj)[0]
    bundle = base + ".hipfb"
    cuid = hashlib.sha1(os.path.abspath(src).encode()).hexdigest()[:16]
    common = ["-x", "hip", *flags(), *EXTRA.get(os.path.basename(src), []), f"-cuid={cuid}"]
    device = [cc, *common, "--offload-device-only", *DEVICE_FLAGS, "-c", src, "-o", bundle]
    host = [cc, *common, "--offload-host-only", "-Xclang", "-fcuda-include-gpubinary",
            "-Xclang", bundle, "-c", src, "-o", obj]
    return [device, host]


def build(verbose: bool = False) -> str:
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objects = []
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        jobs.append(_compile_cmds(cc, os.path.join(CSRC, src), obj))
        objects.append(obj)
    if verbose:
        for job in jobs:
            for cmd in job:
                print(" ".join(cmd), flush=True)

    def run_job(job):
        for cmd in job:
            _run(cmd)

    # the files compile independently: a few at a time
    workers = max(1, min(len(jobs), (os.cpu_count() or 1), 8))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        for f in [pool.submit(run_job, job) for job in jobs]:
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
