"""Builds libcast.so in-tree: every HIP/C++ source under csrc/ compiled by hipcc
for gfx950 and linked into one shared library with a plain C ABI."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcast.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(HERE, "..", "include")]


# Per-file compiler options.  The register sweeps of the batched kernels
# dispatch on a gate's sweep bits to fully unrolled variants that differ only
# in which registers they read; LLVM's sinking of common code would fold the
# variants into one body fed by register copies (16 moves per inner product),
# so it is turned off for that file.
FILE_FLAGS = {"batch_kernels.hip": ["-mllvm", "-simplifycfg-sink-common=false"]}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + FILE_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def _stale(src, headers_mtime):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return t < os.path.getmtime(src) or t < headers_mtime


def build(verbose=False, incremental=False):
    """Compiles every source (or, with incremental, only those whose object
    is older than the source or any header) and links libcast.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    todo = srcs
    if incremental:
        hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
        hdrs.append(os.path.join(HERE, "..", "include", "cast.h"))
        hm = max(os.path.getmtime(h) for h in hdrs)
        todo = [s for s in srcs if _stale(s, hm)]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        results = list(ex.map(_compile, todo))
    results += [(os.path.join(BUILD, os.path.basename(s) + ".o"), "") for s in srcs if s not in todo]
    objs = [o for o, _ in results]
    if verbose:
        for o, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lhiprtc"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


ASAN_DIR = os.path.join(HERE, "_build_asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libcast_asan.so")
ASAN_DRIVER = os.path.join(ASAN_DIR, "host_driver")
# Host code only: hipcc applies each flag after -Xarch_host to the host
# compilation and leaves the gfx950 code as in the normal build.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


# Kernel files whose host side is only launch code; the planning code lives
# in the .cpp files and in diagrun.hip (its schedule builder).
UNSANITIZED = {"apply.hip", "blocked.hip", "batch_kernels.hip", "reduce.hip"}


def build_sanitized(driver_src):
    """A copy of libcast.so whose host planning code (every .cpp source and
    the .hip sources outside UNSANITIZED) is built with AddressSanitizer and
    UndefinedBehaviorSanitizer, and the host driver `driver_src` linked
    against it with the same compiler's runtime (both under _build_asan/).
    Objects are rebuilt only when older than their source or a header.
    Returns the driver's path."""
    os.makedirs(ASAN_DIR, exist_ok=True)
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    hdrs.append(os.path.join(HERE, "..", "include", "cast.h"))
    hm = max(os.path.getmtime(h) for h in hdrs)

    def one(src):
        obj = os.path.join(ASAN_DIR, os.path.basename(src) + ".o")
        if os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(src), hm):
            return obj
        flags = [] if os.path.basename(src) in UNSANITIZED else SANITIZE
        cmd = [HIPCC] + COMMON + flags + ["-c", src, "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized compile failed: {src}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(one, sources()))
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", ASAN_LIB] + SANITIZE + objs +
                       ["-lhiprtc"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitized link failed\n{r.stderr}")
    clangxx = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clangxx):
        clangxx = "/opt/rocm/llvm/bin/clang++"
    r = subprocess.run([clangxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                        "-o", ASAN_DRIVER, driver_src, ASAN_LIB, "-Wl,-rpath," + ASAN_DIR,
                        "-L/opt/rocm/lib", "-lamdhip64", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver link failed\n{r.stderr}")
    return ASAN_DRIVER


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
