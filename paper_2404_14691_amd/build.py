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
HOST_SOURCES = ["sage_api.cpp", "register.cpp", "exec.cpp", "pool.cpp", "util.cpp", "serve.cpp", "exit.cpp",
                "selftest.cpp"]


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


def build_sanitized() -> str:
    """The host self-test driver (csrc/selftest_main.cpp) over the library's
    host sources compiled by g++ with AddressSanitizer and
    UndefinedBehaviorSanitizer; the runtime kernels' object from build()
    is linked unchanged (device code carries no sanitizer).  Returns the
    executable's path (lib/sage_selftest_san)."""
    obj = os.path.join(LIB, "obj")
    krt = os.path.join(obj, "kernels_rt.o")
    if not os.path.exists(krt):
        build()
    san = os.path.join(obj, "san")
    os.makedirs(san, exist_ok=True)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fPIC"]
    jobs, objs = [], []
    for src in HOST_SOURCES + ["selftest_main.cpp"]:
        o = os.path.join(san, src + ".o")
        objs.append(o)
        jobs.append(["g++", *flags, "-c", os.path.join(CSRC, src), "-o", o])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(_run, jobs))
    exe = os.path.join(LIB, "sage_selftest_san")
    _run(["g++", "-fsanitize=address,undefined", *objs, krt, "-o", exe, f"-L{rocm}/lib", f"-Wl,-rpath,{rocm}/lib",
          "-lamdhip64", "-lpthread", "-ldl"])
    return exe


if __name__ == "__main__":
    if "--sanitized" in sys.argv:
        print(build_sanitized())
    else:
        print(build(verbose="-v" in sys.argv))
