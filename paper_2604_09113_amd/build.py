"""Build liblbddc.so (HIP for gfx950) in the package directory.

Each source under csrc/ is compiled by hipcc into _build/ and linked into
paper_2604_09113_amd/liblbddc.so.  The oracle's optional C parts are not part
of this library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbddc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("LBDDC_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I" + os.path.join(HERE, "..", "include")]


# Per-file flags.  The stiffness contraction reads every MFMA result with
# ordinary VALU instructions right away, so its MFMAs write VGPRs directly
# instead of accumulation registers that would first have to be copied out.
EXTRA = {"k_assembly.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def sources():
    return sorted(f for f in os.listdir(SRC) if f.endswith((".hip", ".cpp")))


def _compile(name):
    src = os.path.join(SRC, name)
    obj = os.path.join(OUT, name + ".o")
    cmd = [HIPCC] + FLAGS + EXTRA.get(name, []) + ["-c", src, "-o", obj]
    if name.endswith(".cpp"):
        cmd = [HIPCC] + FLAGS + EXTRA.get(name, []) + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    return name, r.returncode, errs, obj


def build(verbose=False, jobs=None):
    os.makedirs(OUT, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, sources()))
    bad = [r for r in results if r[1] != 0]
    for name, rc, errs, _ in results:
        if errs.strip() and (verbose or rc != 0):
            print(f"--- {name}\n{errs}", file=sys.stderr)
    if bad:
        raise RuntimeError("compile failed: " + ", ".join(b[0] for b in bad))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + [r[3] for r in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
