"""Build libsage.so and the function-body code objects for gfx950.

    python -m paper_2404_14691_amd.build

Outputs (next to this file, in ``lib/``):
  libsage.so          runtime + fingerprint / block-copy kernels + C ABI
  sage_mlp.hsaco      MLP bodies, loaded with hipModuleLoad by fn_register
  sage_stencil.hsaco  stencil body, loaded the same way
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "lib")
ARCH = "gfx950"


def hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if p and os.path.exists(p):
            return p
    raise RuntimeError("hipcc not found")


# packed FP32 instructions are disabled for every device compile
DEVICE_FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_SOURCES = ["sage_api.cpp", "register.cpp", "exec.cpp", "pool.cpp", "util.cpp", "serve.cpp", "exit.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(LIB, exist_ok=True)
    obj = os.path.join(LIB, "obj")
    os.makedirs(obj, exist_ok=True)
    cc = hipcc()
    jobs = []
    objs = []
    for src in HOST_SOURCES:
        if not os.path.exists(os.path.join(CSRC, src)):
            continue
        o = os.path.join(obj, src + ".o")
        objs.append(o)
        jobs.append([cc, *DEVICE_FLAGS, "-fPIC", "-fvisibility=hidden", "-Wall", "-Wno-unused-result", "-c",
                     os.path.join(CSRC, src), "-o", o])
    o = os.path.join(obj, "kernels_rt.o")
    objs.append(o)
    jobs.append([cc, *DEVICE_FLAGS, "-fPIC", "-fvisibility=hidden", "-c", os.path.join(CSRC, "kernels_rt.hip"), "-o", o])
    for name, src in (("sage_mlp.hsaco", "body_mlp.hip"), ("sage_stencil.hsaco", "body_stencil.hip")):
        jobs.append([cc, *DEVICE_FLAGS, "--genco", os.path.join(CSRC, src), "-o", os.path.join(LIB, name)])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    tmp = os.path.join(LIB, "libsage.so.tmp")
    outs.append(_run([cc, *DEVICE_FLAGS, "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread", "-ldl"]))
    os.replace(tmp, os.path.join(LIB, "libsage.so"))
    if verbose:
        for s in outs:
            if s.strip():
                print(s)
    return os.path.join(LIB, "libsage.so")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
