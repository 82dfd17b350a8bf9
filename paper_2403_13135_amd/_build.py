"""Build ``libsil.so`` (gfx950) in-tree with hipcc."""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libsil.so")
SOURCES = [os.path.join(PKG, "csrc", n) for n in ("sil.hip", "label_ex.hip", "server.cpp", "unet.hip")]
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _run(cmd):
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)


def _messages(text: str):
    # hipcc's host pass does not know the packed-fp32 feature; drop that notice
    noise = "is not a recognized feature for this target"
    return [l for l in text.splitlines() if noise not in l]


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compile every source to an object in parallel, then link the library."""
    os.makedirs(OBJDIR, exist_ok=True)
    compile_flags = [f for f in HIP_FLAGS if f != "-shared"]
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        cmd = [HIPCC, *compile_flags, *extra_flags, "-I", INCLUDE, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        objs.append(obj)
        procs.append((src, _run(cmd)))
    errors = []
    for src, proc in procs:
        out, _ = proc.communicate()
        msgs = _messages(out)
        if proc.returncode != 0:
            errors.append(f"{os.path.basename(src)}:\n" + "\n".join(msgs))
        elif verbose and msgs:
            print("\n".join(msgs), flush=True)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *HIP_FLAGS, *extra_flags, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + "\n".join(_messages(res.stdout + res.stderr)))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
