"""Build libsv.so (HIP for gfx950) in-tree.

    python -m paper_2608_09733_amd.build

hipcc flags:
  -Xclang -target-feature -Xclang -packed-fp32-ops   no packed FP32 instructions
  -mllvm -simplifycfg-sink-common=false              keep per-target switch arms
      apart, so register groups stay in VGPRs (common-code sinking turns the
      compile-time slot indices into dynamic ones and demotes groups to scratch)
"""
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsv.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-simplifycfg-sink-common=false",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


def _variants_text():
    return open(os.path.join(CSRC, "sv_variants.h")).read()


def variants():
    """(T, M, R, NS) entries of SVI_VARIANTS in sv_variants.h."""
    return re.findall(r"X\((double|float),\s*(\d+),\s*(\d+),\s*(\d+)\)", _variants_text())


def batch_variants():
    """(T, M, R) entries of SVB_VARIANTS in sv_variants.h."""
    txt = _variants_text()
    txt = txt[txt.index("#define SVB_VARIANTS"):]
    return re.findall(r"X\((double|float),\s*(\d+),\s*(\d+)\)", txt)


def build(verbose: bool = False, jobs: int = 0) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    todo = []
    for src in ["sv_kernels.hip", "sv_host.cpp"]:
        obj = os.path.join(objdir, src + ".o")
        cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC, "-x", "hip"] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
        todo.append((cmd, obj))
    for t, m, r, ns in variants():
        obj = os.path.join(objdir, f"sweep_{t}_{m}_{r}_{ns}.o")
        cmd = [HIPCC] + COMMON + [f"-DSVI_VT={t}", f"-DSVI_VM={m}", f"-DSVI_VR={r}",
                                  f"-DSVI_VNS={ns}", "-c",
                                  os.path.join(CSRC, "sv_sweep_variant.hip"), "-o", obj]
        todo.append((cmd, obj))
    for t, m, r in batch_variants():
        obj = os.path.join(objdir, f"batch_{t}_{m}_{r}.o")
        cmd = [HIPCC] + COMMON + [f"-DSVB_VT={t}", f"-DSVB_VM={m}", f"-DSVB_VR={r}", "-c",
                                  os.path.join(CSRC, "sv_batch_variant.hip"), "-o", obj]
        todo.append((cmd, obj))
    # longest jobs first
    todo.sort(key=lambda j: 0 if "sv_batch_variant" in " ".join(j[0]) else 1)
    objs = [o for _, o in todo]
    running = []
    while todo or running:
        while todo and len(running) < jobs:
            cmd, _ = todo.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                  stderr=subprocess.STDOUT, text=True)))
        cmd, p = running.pop(0)
        out, _ = p.communicate()
        out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            for _, q in running:
                q.kill()
            raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    tmp = LIB + ".tmp"
    for f in os.listdir(objdir):
        if f.endswith(".o") and os.path.join(objdir, f) not in objs:
            os.remove(os.path.join(objdir, f))
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
