"""Build the HIP library libmera.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["contract.hip", "contract_b3.hip", "contract_b3x.hip", "aux.hip", "peak.hip", "symeig.hip", "mera_api.hip"]
LIB = os.path.join(HERE, "libmera.so")

# Packed-FP32 instructions are disabled: the compiler must not form v_pk_*_f32 from float code.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in VGPRs: avoids AGPR<->VGPR copies around the k loop
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


# Host-side sanitizers for the CPU checks of the planner, argument checks and sizing code
# (libmera_asan.so; never loaded on a GPU: the device code is built without them).
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer"]
LIB_ASAN = os.path.join(HERE, "libmera_asan.so")


def build(verbose: bool = False, jobs: int = 8, sanitize: bool = False, out_dir: str | None = None) -> str:
    """Compile every source and link the library; returns its path.

    `sanitize` builds the host code with AddressSanitizer and UBSan (libmera_asan.so);
    `out_dir` puts the objects and the library there instead of the package directory.
    """
    lib = LIB_ASAN if sanitize else LIB
    objdir = os.path.join(HERE, "_build_asan" if sanitize else "_build")
    if out_dir is not None:
        lib = os.path.join(out_dir, os.path.basename(lib))
        objdir = os.path.join(out_dir, os.path.basename(objdir))
    os.makedirs(objdir, exist_ok=True)
    extra = SANITIZE_FLAGS if sanitize else []
    objs = [os.path.join(objdir, src.replace(".hip", ".o")) for src in SOURCES]
    pending = list(zip(SOURCES, objs))
    running = []
    failed = []

    def finish(src, p):
        out, _ = p.communicate()
        lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed.append(src)
            print("\n".join(lines), file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))

    # at most `jobs` compilers at a time
    while pending or running:
        while pending and len(running) < max(1, jobs):
            src, obj = pending.pop(0)
            cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                  text=True)))
        finish(*running.pop(0))
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = lib + ".tmp"
    link = ["-shared-libsan", *extra] if sanitize else []
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *link, *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
