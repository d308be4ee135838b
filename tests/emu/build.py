"""Builds the host emulation of libtpx (test infrastructure): the library's
HIP sources compiled unchanged by g++ against tests/emu/hip_emu.h, with
AddressSanitizer and UndefinedBehaviorSanitizer, into one executable.  The
build is the bounds-checked build of the kernels: every global and LDS access
of an emulated kernel is checked by the sanitizers."""
from __future__ import annotations

import concurrent.futures
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2603_04942_amd", "csrc")
OUT_DIR = os.path.join(HERE, "_build")
EXE = os.path.join(OUT_DIR, "emu_tpx")
HIP_SOURCES = ["tpx_decode.hip", "tpx_cluster.hip", "tpx_util.hip", "tpx_api.hip",
               "tpx_service.hip"]
FLAGS = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-I", os.path.join(HERE, "include"),
         "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable"]


def _inputs():
    files = [os.path.join(CSRC, s) for s in HIP_SOURCES]
    files += [os.path.join(CSRC, h) for h in ("tpx_internal.h", "tpx_kernels.h",
                                              "tpx_decode_dev.h", "tpx_util_dev.h")]
    files += [os.path.join(ROOT, "include", "tpx.h")]
    files += [os.path.join(HERE, f) for f in ("hip_emu.h", "hip_emu.cpp", "emu_main.cpp",
                                               "emu_selftest.cpp", "build.py")]
    return files


def _digest():
    h = hashlib.sha256()
    for f in _inputs():
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _compile(args):
    src, obj, lang = args
    cmd = ["g++", *FLAGS, "-x", lang, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"emulation build failed on {src}:\n{r.stderr[-6000:]}")
    return obj


def build(force: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    stamp = os.path.join(OUT_DIR, "stamp")
    dig = _digest()
    if not force and os.path.exists(EXE) and os.path.exists(stamp):
        with open(stamp) as f:
            if f.read() == dig:
                return EXE
    jobs = [(os.path.join(CSRC, s), os.path.join(OUT_DIR, s + ".o"), "c++") for s in HIP_SOURCES]
    jobs += [(os.path.join(HERE, s), os.path.join(OUT_DIR, s + ".o"), "c++")
             for s in ("hip_emu.cpp", "emu_main.cpp", "emu_selftest.cpp")]
    with concurrent.futures.ThreadPoolExecutor(min(8, len(jobs))) as ex:
        objs = list(ex.map(_compile, jobs))
    tmp = EXE + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", *FLAGS, *objs, "-o", tmp, "-lpthread"])
    os.replace(tmp, EXE)
    with open(stamp, "w") as f:
        f.write(dig)
    return EXE


if __name__ == "__main__":
    print(build(force=True))
