"""Build the HIP library liblpic.so for gfx950 in-tree (hipcc, no JIT).

The translation units compile in parallel into objects in a temporary folder, then
link into the shared library; the library is replaced only once the link succeeds."""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "liblpic.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("lpic_kernels.hip", "lpic_fused.hip", "lpic_qed.hip", "lpic_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("lpic_device.hpp", "lpic_internal.hpp")] + \
          [os.path.join(ROOT, "include", "lpic.h")]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-munsafe-fp-atomics",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def _clean(stderr):
    return "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l)


def build(verbose=False, out=SO, defines=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include")] + [f"-D{d}" for d in defines]
    with tempfile.TemporaryDirectory(prefix="lpic_build_") as tmp:
        procs = []
        for src in SOURCES:
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            cmd = [hipcc, *FLAGS, *inc, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((obj, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.PIPE, text=True)))
        objs, errs = [], []
        for obj, p in procs:
            _, err = p.communicate()
            if p.returncode != 0:
                errs.append(f"hipcc failed ({p.returncode}):\n{_clean(err)}")
            elif _clean(err).strip() and verbose:
                print(_clean(err), file=sys.stderr)
            objs.append(obj)
        if errs:
            raise RuntimeError("\n".join(errs))
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out + ".tmp", *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed ({res.returncode}):\n{_clean(res.stderr)}")
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
