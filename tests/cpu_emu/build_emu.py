"""Build the library's sources for the CPU emulation (hip/hip_runtime.h here) with
AddressSanitizer, linked with emu_driver.cpp into one executable.  Test infrastructure only:
the sources are copied under _build/ as C++ files (the same text) and compiled with g++;
the result is cached by the sources' hash."""
import hashlib
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.abspath(os.path.join(HERE, "..", ".."))
CSRC = os.path.join(ROOT, "paper_2403_03156_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["fsmp_api.hip", "fsmp_kernels.hip", "fsmp_server.hip"]
HEADERS = ["fsmp_internal.h"]
FLAGS = ["-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-pthread",
         "-Wno-attributes", "-Wno-unused-variable", "-Wno-unused-function"]


def _hash(csrc):
    h = hashlib.sha256()
    for f in [os.path.join(csrc, s) for s in SOURCES + HEADERS] + [os.path.join(INCLUDE, "fsmp.h"),
                                                                   os.path.join(HERE, "hip", "hip_runtime.h"),
                                                                   os.path.join(HERE, "emu_driver.cpp")]:
        h.update(open(f, "rb").read())
    h.update(" ".join(FLAGS).encode())
    return h.hexdigest()[:16]


def build(verbose=False, csrc=CSRC, build_dir=BUILD):
    """Path of the emulation driver, compiled if the sources changed (csrc: the directory of
    the library's sources, build_dir: where to build, emptied first)."""
    tag = _hash(csrc)
    exe = os.path.join(build_dir, f"emu_driver_{tag}")
    if os.path.exists(exe):
        return exe
    if os.path.isdir(build_dir):
        shutil.rmtree(build_dir)
    src = os.path.join(build_dir, "src", "csrc")
    os.makedirs(src)
    os.makedirs(os.path.join(build_dir, "include"))
    # the sources include "../../include/fsmp.h" relative to their own directory
    shutil.copy(os.path.join(INCLUDE, "fsmp.h"), os.path.join(build_dir, "include", "fsmp.h"))
    for h in HEADERS:
        shutil.copy(os.path.join(csrc, h), os.path.join(src, h))
    objs = []
    jobs = []
    for s in SOURCES:
        cpp = os.path.join(src, s.replace(".hip", ".cpp"))
        shutil.copy(os.path.join(csrc, s), cpp)
        obj = cpp[:-4] + ".o"
        cmd = ["g++", *FLAGS, "-I", HERE, "-c", cpp, "-o", obj]
        jobs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    drv = os.path.join(build_dir, "emu_driver.o")
    jobs.append(subprocess.Popen(["g++", *FLAGS, "-I", HERE, "-I", os.path.join(build_dir, "include"), "-c",
                                  os.path.join(HERE, "emu_driver.cpp"), "-o", drv],
                                 stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for j in jobs:
        out, _ = j.communicate()
        if j.returncode != 0:
            raise RuntimeError("CPU emulation build failed:\n" + out.decode()[-4000:])
        if verbose and out:
            print(out.decode()[-2000:])
    subprocess.check_call(["g++", *FLAGS, *objs, drv, "-o", exe + ".tmp"])
    os.replace(exe + ".tmp", exe)
    return exe


if __name__ == "__main__":
    print(build(verbose=True))
