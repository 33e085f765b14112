"""Build the HIP shared library libdd.so in-tree for gfx950.

    python -m paper_2205_11638_amd.build      (or call build())

Host C++ is compiled with g++, device code with hipcc --offload-arch=gfx950; the
objects are linked by hipcc into paper_2205_11638_amd/libdd.so.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdd.so")
# host-side AddressSanitizer / UndefinedBehaviorSanitizer build (CPU checks of the diagram compiler and
# the host logic; device code is built as usual)
LIB_SAN = os.path.join(HERE, "libdd_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-O1", "-g"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HOST_SRC = ["bdd.cpp", "dd_api.cpp", "batch.cpp", "autotune.cpp"]
DEVICE_SRC = ["kernels.hip", "adjoint.hip", "features.hip", "noalloc.hip"]
# packed-fp32 instructions are disabled for all device code
# -fno-honor-nans: the solver never forms NaN (infinite costs only mark 0-terminal arcs and
# are never subtracted), so min/max need no NaN-quieting; parameter checks use bit tests.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-fno-honor-nans", "-Wall", "-Wno-unused-result"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]
# device objects of the last build, keyed by the sources and flags they came from: the sanitized
# build (host objects only differ) links them instead of compiling the device code again
OBJ_CACHE = os.path.join(HERE, "_objcache")


def _device_key():
    h = hashlib.sha256(" ".join(HIP_FLAGS).encode())
    for d, names in ((CSRC, sorted(os.listdir(CSRC))), (os.path.join(HERE, "..", "include"), ["dd.h"])):
        for f in names:
            if f.endswith((".hip", ".hpp", ".cpp", ".h")):
                h.update(f.encode())
                h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:24]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} ({r.returncode})")
    return r


def build(verbose=False, sanitize=False) -> str:
    """Compile every source (always) and link libdd.so (libdd_san.so with sanitize: host objects built
    with ASan/UBSan, for CPU-only checks); returns the library path."""
    out_lib = LIB_SAN if sanitize else LIB
    host_flags = HOST_FLAGS + (SAN_FLAGS if sanitize else [])
    key = _device_key()
    cached = os.path.join(OBJ_CACHE, key)
    reuse = sanitize and all(os.path.exists(os.path.join(cached, f + ".o")) for f in DEVICE_SRC)
    with tempfile.TemporaryDirectory(prefix="ddbuild") as tmp:
        objs = []
        procs = []
        for f in HOST_SRC:
            o = os.path.join(tmp, f + ".o")
            procs.append((["g++", *host_flags, "-c", os.path.join(CSRC, f), "-o", o]))
            objs.append(o)
        for f in DEVICE_SRC:
            if reuse:
                objs.append(os.path.join(cached, f + ".o"))
                continue
            o = os.path.join(tmp, f + ".o")
            procs.append(([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, f), "-o", o]))
            objs.append(o)
        running = [(c, subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
                   for c in procs]
        for c, p in running:
            out, _ = p.communicate()
            if verbose and out:
                sys.stderr.write(out)
            if p.returncode != 0:
                sys.stderr.write(" ".join(c) + "\n" + (out or ""))
                raise RuntimeError("compile failed: " + c[-3])
        tmp_lib = out_lib + ".tmp%d" % os.getpid()
        # with sanitize the runtimes of the g++-built host objects are left unresolved here: the checking
        # process preloads gcc's libasan and libubsan
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib, *objs, "-lpthread"])
        os.replace(tmp_lib, out_lib)
        if not reuse:  # keep this build's device objects (only the latest key)
            shutil.rmtree(OBJ_CACHE, ignore_errors=True)
            os.makedirs(cached, exist_ok=True)
            for f in DEVICE_SRC:
                shutil.copy(os.path.join(tmp, f + ".o"), os.path.join(cached, f + ".o"))
    return out_lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
