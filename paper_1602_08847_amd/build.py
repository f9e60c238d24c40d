"""Build libmuffin.so for gfx950 in-tree with hipcc (one shared library, C ABI in include/muffin.h)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["api.hip", "fft.hip", "iuwt.hip", "spectral.hip", "reduce.hip", "cnn.hip", "uob.hip", "vis.hip"]
LIB = os.path.join(HERE, "libmuffin.so")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _compile_and_link(extra: list, objdir: str, lib: str, verbose: bool) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for s in SOURCES:
        obj = os.path.join(objdir, s.replace(".hip", ".o"))
        cmd = [hipcc, *FLAGS, *extra, "-c", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               os.path.join(CSRC, s), "-o", obj]
        cmd.remove("-shared")
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if verbose and lines:
            print(f"[{s}]\n" + "\n".join(lines[-40:]))
        if p.returncode != 0:
            failed.append(s)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = lib + ".tmp"
    cmd = [hipcc, *FLAGS, *extra, *objs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = True, jobs: int = 8) -> str:
    return _compile_and_link([], os.path.join(HERE, "_build"), LIB, verbose)


CHECKED_LIB = os.path.join(HERE, "libmuffin_checked.so")  # in-tree: it ships with the package


def build_checked(verbose: bool = True) -> str:
    """The same library with MF_CHECKED: instrumented kernel indices are bounds-checked on the
    device (a miss is counted and replaced by an index in bounds; muffin_debug_oob reads the count).
    Test infrastructure: the GPU tests load it through MUFFIN_LIBRARY."""
    return _compile_and_link(["-DMF_CHECKED"], os.path.join(HERE, "_build", "checked"), CHECKED_LIB, verbose)


# Host code under AddressSanitizer and UndefinedBehaviorSanitizer (device code is not
# instrumented: each sanitizer flag applies to the host compilation only).
HOST_SANITIZERS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def build_host_sanitized(verbose: bool = False) -> str:
    """libmuffin with its host code built with ASan and UBSan (device code as usual, at -O1), and
    the host check driver tests/host_sanitizer_driver.cpp linked against it; returns the driver."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    outdir = os.path.join(HERE, "_build", "hostsan")
    os.makedirs(outdir, exist_ok=True)
    base = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
            "-packed-fp32-ops", "-Wno-unused-result", *HOST_SANITIZERS]
    procs, objs = [], []
    for s in SOURCES:
        obj = os.path.join(outdir, s.replace(".hip", ".o"))
        cmd = [hipcc, *base, "-c", "-I", os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(CSRC, s), "-o", obj]
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    for s, pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError(f"hipcc (host sanitizers) failed for {s}:\n" + out.decode(errors="replace")[-4000:])
    lib = os.path.join(outdir, "libmuffin_hostsan.so")
    r = subprocess.run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *HOST_SANITIZERS, *objs, "-o", lib],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link (host sanitizers) failed:\n" + r.stdout.decode(errors="replace")[-4000:])
    exe = os.path.join(outdir, "host_sanitizer_driver")
    drv = os.path.join(ROOT, "tests", "host_sanitizer_driver.cpp")
    dobj = os.path.join(outdir, "host_sanitizer_driver.o")
    r = subprocess.run([hipcc, *base, "-I", os.path.join(ROOT, "include"), "-c", drv, "-o", dobj],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode == 0:
        r = subprocess.run([hipcc, *HOST_SANITIZERS, dobj, lib, "-Wl,-rpath," + outdir, "-o", exe],
                           stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("driver build failed:\n" + r.stdout.decode(errors="replace")[-4000:])
    if verbose:
        print(exe)
    return exe


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
