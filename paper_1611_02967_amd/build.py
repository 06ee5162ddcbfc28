"""Compiles libchhs.so (HIP, gfx950) in-tree with hipcc.

The library is a plain C ABI (``include/chhs.h``); no PyTorch extension is
involved.  Every translation unit is compiled to an object in parallel and
linked into ``paper_1611_02967_amd/libchhs.so``.  Next to it, ``libchhs.so.sha256``
records the digest of the sources, the header and the compiler flags it was
built from; the binding refuses a library whose digest no longer matches.
"""
import hashlib
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libchhs.so")
STAMP = LIB + ".sha256"
ARCH = "gfx950"

SOURCES = ["chhs_api.hip", "chhs_kernels.hip", "chhs_tile2d.hip", "chhs_stream2d.hip",
           "chhs_tail.hip", "chhs_noalloc.hip", "chhs_refine2d.hip",
           "chhs_step3d.hip", "chhs_resid3d.hip"]

# -packed-fp32-ops: keep the compiler from forming packed FP32 instructions
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]


def source_digest(defines=()):
    """sha256 over every file of csrc/, the public header and the build flags."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    with open(os.path.join(INCLUDE, "chhs.h"), "rb") as fh:
        h.update(fh.read())
    # flags without the include directories (absolute paths differ between
    # copies of the tree)
    flags = [f for f in COMMON if not f.startswith("-I")] + [f"-D{d}" for d in defines]
    h.update(" ".join(flags).encode())
    return h.hexdigest()


def is_current(path=LIB):
    """True if ``path`` exists and was built from the sources as they are now."""
    try:
        with open(path + ".sha256") as fh:
            return os.path.exists(path) and fh.read().strip() == source_digest()
    except OSError:
        return False


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose=False, out=None, defines=()):
    """Compile every source and link libchhs.so (or ``out``, with extra -D
    ``defines`` for kernel variants); raises on any compiler error."""
    cc = hipcc()
    target = out or LIB
    with tempfile.TemporaryDirectory(prefix="chhs_build_") as tmp:
        def compile_one(src):
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            cmd = [cc, *COMMON, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
            return obj
        with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        out_tmp = os.path.join(tmp, "libchhs.so")
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        shutil.copyfile(out_tmp, target + ".tmp")
        os.replace(target + ".tmp", target)
        with open(target + ".sha256.tmp", "w") as fh:
            fh.write(source_digest(defines) + "\n")
        os.replace(target + ".sha256.tmp", target + ".sha256")
    return target


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
