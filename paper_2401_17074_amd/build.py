"""Build libtslb.so for gfx950 with hipcc (in-tree, no JIT cache)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["capi.hip", "aux_kernels.hip", "update_direct.hip", "update_tiled.hip", "adjoint_tiled.hip",
           "update_poplayout.hip", "stats.hip",
           "update_d2q9.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC", "-Wall",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False, defines=()):
    """Compile and link libtslb.so (all sources in parallel).  `defines`
    (e.g. ("TSLB_NT_STORE=0", "TSLB_WAVES_PER_EU=3")) are build-time tuning
    overrides of the tiled kernels."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj_dir = os.path.join(ROOT, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(obj_dir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc] + FLAGS + ["-D" + d for d in defines] + ["-c", os.path.join(HERE, "csrc", src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for cmd, p in procs:
        out, _ = p.communicate()
        text = "\n".join(ln for ln in out.decode(errors="replace").splitlines()
                         if "packed-fp32-ops" not in ln)
        if p.returncode != 0:
            failed.append((cmd, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        for cmd, text in failed:
            sys.stderr.write(" ".join(cmd) + "\n" + text + "\n")
        raise RuntimeError("hipcc failed")
    lib = os.path.join(HERE, "libtslb.so")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", lib + ".tmp"])
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, defines=tuple(sys.argv[1:]))
