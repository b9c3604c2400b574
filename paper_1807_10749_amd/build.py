"""Compile the HIP/C++ sources into paper_1807_10749_amd/libsfpath.so for gfx950."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsfpath.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["kernels.hip", "noalloc.hip", "planner.cpp", "executor.cpp", "sfpath.cpp", "server.cpp", "jit.cpp"]
# device headers the run-time compiled pass kernels include (jit.cpp), built into the library
JIT_HEADERS = ["sf_device.hpp", "pass_dev.hpp"]


def write_jit_headers() -> str:
    """Writes _build/jit_headers.cpp: the JIT_HEADERS' text as string constants."""
    out = os.path.join(BUILD, "jit_headers.cpp")
    names, texts = [], []
    for h in JIT_HEADERS:
        with open(os.path.join(CSRC, h)) as f:
            text = f.read()
        if ")SFJIT\"" in text:
            raise RuntimeError(h + " holds the raw-string delimiter")
        names.append('"' + h + '"')
        texts.append('R"SFJIT(' + text + ')SFJIT"')
    src = ("namespace sf {\nextern const char *const kJitHeaderNames[2];\nextern const char *const kJitHeaderText[2];\n"
           "const char *const kJitHeaderNames[2] = {" + ", ".join(names) + "};\n"
           "const char *const kJitHeaderText[2] = {\n" + ",\n".join(texts) + "};\n}  // namespace sf\n")
    old = open(out).read() if os.path.exists(out) else None
    if old != src:
        with open(out, "w") as f:
            f.write(src)
    return out
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(HERE, "..", "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES + ["jit_headers.cpp"]:
        path = write_jit_headers() if src == "jit_headers.cpp" else os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        if src.endswith(".hip"):
            cmd = [HIPCC, "-x", "hip", *DEVICE, *COMMON, "-c", path, "-o", obj]
        else:
            cmd = ["g++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *COMMON, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            if procs.pop(0).wait():
                raise RuntimeError("compile failed")
    for p in procs:
        if p.wait():
            raise RuntimeError("compile failed")
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lhiprtc"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
