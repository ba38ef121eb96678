"""Build the gfx950 HIP library libspg.so in-tree with hipcc.

Usage: python -m paper_1905_13408_amd.build            (or build() from Python)
       python -m paper_1905_13408_amd.build --sanitized (host ASan + UBSan build, see below)

The two sources compile to objects under _build/ in parallel, then link into libspg.so.
build_sanitized() links the same kernel object with the host runtime (validation, workspace
carving, launch sequence) recompiled under the host address and undefined-behaviour
sanitizers into libspg_san.so: GPU code is never built with a sanitizer.  That library loads
only with the sanitizer runtime preloaded (sanitizer_runtime()); the binding picks it up
through SPG_LIB_PATH.
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
KERNELS = os.path.join(CSRC, "spg_kernels.hip")
API = os.path.join(CSRC, "spg_api.hip")
LIB = os.path.join(HERE, "libspg.so")
LIB_SAN = os.path.join(HERE, "libspg_san.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed fp32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]
# host-side sanitizers only: each -fsanitize= applies to the host compilation
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _run_all(cmds):
    procs = [subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True) for c in cmds]
    for c, p in zip(cmds, procs):
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out + err)
            raise RuntimeError(f"hipcc failed: {' '.join(c[-3:])}")


def _compile(src, obj, extra=()):
    return [HIPCC] + FLAGS + list(extra) + ["-c", src, "-o", obj]


def _link(objs, out, extra=()):
    tmp = out + ".tmp"
    _run_all([[HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + list(extra) + ["-o", tmp] + objs])
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Compile both sources (always) and link libspg.so."""
    os.makedirs(OBJ, exist_ok=True)
    ko, ao = os.path.join(OBJ, "spg_kernels.o"), os.path.join(OBJ, "spg_api.o")
    _run_all([_compile(KERNELS, ko), _compile(API, ao)])
    return _link([ko, ao], LIB)


def build_sanitized() -> str:
    """libspg_san.so: the kernel object of the last build() (compiled if missing or older than
    its sources) and the host runtime under ASan + UBSan."""
    os.makedirs(OBJ, exist_ok=True)
    ko, so = os.path.join(OBJ, "spg_kernels.o"), os.path.join(OBJ, "spg_api_san.o")
    deps = [KERNELS, os.path.join(CSRC, "spg_internal.h")]
    cmds = [_compile(API, so, SAN_FLAGS + ["-O1", "-g"])]
    if not os.path.exists(ko) or os.path.getmtime(ko) < max(os.path.getmtime(d) for d in deps):
        cmds.append(_compile(KERNELS, ko))
    _run_all(cmds)
    return _link([ko, so], LIB_SAN, ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"])


def sanitizer_runtime() -> str:
    """Path of the host ASan runtime shared library of the toolchain (preloaded to load
    libspg_san.so into an unsanitized interpreter)."""
    root = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    hits = sorted(glob.glob(os.path.join(root, "lib", "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")) +
                  glob.glob(os.path.join(root, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("no libclang_rt.asan-x86_64.so next to hipcc")
    return hits[-1]


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--sanitized":
        print(build_sanitized())
    else:
        print(build(verbose=True))
