"""Compile libmnufft.so (HIP kernels + C ABI) for gfx950 with hipcc.

Objects go to ``_build/`` next to this file and are compiled in parallel; the
shared library is written in-tree as ``libmnufft.so`` so that it travels with
the source tree.  ``build()`` always recompiles.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmnufft.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
    # packed FP32 instructions are kept out of the generated code on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", f"-I{INCLUDE}",
]

# (source, extra flags, object name)
UNITS = [
    ("mnufft.cpp", [], "mnufft.o"),
    ("host_common.cpp", [], "host_common.o"),
    ("batch.cpp", [], "batch.o"),
    ("tune.cpp", [], "tune.o"),
    ("select.cpp", [], "select.o"),
    ("kernels_mlp.hip", [], "kernels_mlp.o"),
    ("kernels_sort.hip", [], "kernels_sort.o"),
    ("kernels_deconv.hip", [], "kernels_deconv.o"),
    ("kernels_type3.hip", [], "kernels_type3.o"),
    ("spread_dispatch.hip", [], "spread_dispatch.o"),
    ("spread_inst.hip", ["-DMN_T=float", "-DMN_D=1"], "spread_f1.o"),
    ("spread_inst.hip", ["-DMN_T=double", "-DMN_D=1"], "spread_d1.o"),
    ("spread_inst.hip", ["-DMN_T=float", "-DMN_D=2"], "spread_f2.o"),
    ("spread_inst.hip", ["-DMN_T=float", "-DMN_D=3"], "spread_f3.o"),
    ("spread_inst.hip", ["-DMN_T=double", "-DMN_D=2"], "spread_d2.o"),
    ("spread_inst.hip", ["-DMN_T=double", "-DMN_D=3"], "spread_d3.o"),
]


def _compile(unit):
    src, extra, obj = unit
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC] + COMMON + extra + lang + ["-c", os.path.join(CSRC, src), "-o",
                                            os.path.join(OUT, obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    return r.returncode, " ".join(cmd), "\n".join(msgs)


def build(jobs=None, verbose=False):
    """Compile every unit and link ``libmnufft.so``; raises on failure."""
    os.makedirs(OUT, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, UNITS))
    failed = [(cmd, msg) for rc, cmd, msg in results if rc != 0]
    for rc, cmd, msg in results:
        if verbose and msg.strip():
            print(msg, file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n\n".join(f"{c}\n{m}" for c, m in failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
        [os.path.join(OUT, u[2]) for u in UNITS] + ["-lrocfft"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
