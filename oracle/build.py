"""Compile the oracle's C source into a shared library for this host (gcc, OpenMP).

The library is built with -O3 -march=native, so a build is only valid on the
CPU it was made on: its file name carries a hash of this machine's CPU model
and instruction-set flags (``liboracle-<hash>.so``), and a machine that finds
no library of its own builds one (a few seconds of gcc).  -ffp-contract=off
keeps every product and sum rounded on its own (no fused multiply-add), as the
acceptance decisions of rejection sampling are defined, so the native build
computes the same values as a generic one.
"""
import hashlib
import os
import platform
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sf_oracle.c")

FLAGS = ["-std=gnu11", "-O3", "-march=native", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
         "-Wall", "-Wextra", "-Wno-unused-parameter"]


def cpu_tag() -> str:
    """Short hash of this host's CPU model and flags (what -march=native depends on)."""
    info = platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            model = flags = ""
            for line in f:
                if line.startswith("model name") and not model:
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("flags") and not flags:
                    flags = " ".join(sorted(line.split(":", 1)[1].split()))
            info += "|" + model + "|" + flags
    except OSError:
        pass
    return hashlib.sha256(info.encode()).hexdigest()[:12]


def out_path() -> str:
    return os.path.join(HERE, f"liboracle-{cpu_tag()}.so")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def build(verbose: bool = False) -> str:
    out = out_path()
    tmp = f"{out}.tmp{os.getpid()}"
    cmd = ["gcc", *FLAGS, "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
