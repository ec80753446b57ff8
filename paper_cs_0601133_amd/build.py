"""Build libffgemm.so (HIP, gfx950) in-tree.

Every source under csrc/ is compiled by hipcc for gfx950 into _build/ and
linked into paper_cs_0601133_amd/libffgemm.so.  ``build()`` always
recompiles (it is the "does it build" check); ``ensure_built()`` only builds
when the library is missing.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libffgemm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # keep the compiler away from packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-pass-failed", "-I", CSRC]


# Per-source flags.  The FP64 kernels fold their accumulators with vector
# ALU code between matrix-core steps; with accumulators in AGPRs the
# compiler would move all of them to VGPRs and back around every fold.
PER_FILE = {"kernels_f64.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
            # the LQUP panel's walk over its 64 rows must unroll completely so
            # that each thread's column stays in registers
            "kernels_lqup.hip": ["-mllvm", "-pragma-unroll-threshold=1000000"],
            # likewise the 64-step walk of the diagonal-block inverse, whose
            # next step's coefficients are requested a step ahead
            "kernels_trsm.hip": ["-mllvm", "-pragma-unroll-threshold=1000000"]}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src, out_dir=OUT, defines=()):
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + PER_FILE.get(os.path.basename(src), []) + \
        [f"-D{d}" for d in defines] + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(jobs=None, defines=(), lib=LIB, out_dir=OUT):
    """Compile every source and link lib.  defines: extra -D flags (kernel
    experiments build into a separate out_dir/lib)."""
    os.makedirs(out_dir, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, out_dir, defines), sources()))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + \
        ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


def ensure_built():
    if not os.path.exists(LIB):
        build()
    return LIB


if __name__ == "__main__":
    print(build())
