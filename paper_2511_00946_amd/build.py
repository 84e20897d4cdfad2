"""Build the HIP library libkkt.so for gfx950 (in-tree, next to this file).

The host plan and dense kernels (kkt.hip) and the row-lane kernels of each
block class (kkt_wave_inst.hip, once per class) compile in parallel to objects
that are linked into one shared library."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libkkt.so")
BUILD = os.path.join(HERE, "_build")
WAVE_CLASSES = (8, 16, 24, 32, 48)

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _units():
    units = [("kkt", os.path.join(CSRC, "kkt.hip"), []), ("kkt_ragged", os.path.join(CSRC, "kkt_ragged.hip"), []),
             ("kkt_qp", os.path.join(CSRC, "kkt_qp.hip"), [])]
    for bp in WAVE_CLASSES:
        # single-wave classes: one instance per right-hand-side count
        for nr in ((1, 4, 8) if bp <= 16 else (8,)):
            units.append(("kkt_wave%d_%d" % (bp, nr), os.path.join(CSRC, "kkt_wave_inst.hip"),
                          ["-DKKT_WAVE_BP=%d" % bp, "-DKKT_WAVE_NR=%d" % nr]))
    return units


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    return res.returncode, out


def build(verbose=False, extra_flags=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    jobs = []
    for name, src, defs in _units():
        obj = os.path.join(BUILD, name + ".o")
        jobs.append((obj, [hipcc] + HIPCC_FLAGS + list(extra_flags) + inc + defs + ["-c", "-o", obj, src]))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "8"))))
    with ThreadPoolExecutor(workers) as pool:
        results = list(pool.map(lambda j: _run(j[1], verbose), jobs))
    for (obj, _), (rc, out) in zip(jobs, results):
        if rc != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (obj, out))
    tmp = OUT + ".tmp%d" % os.getpid()
    rc, out = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in jobs], verbose)
    if rc != 0:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise RuntimeError("link failed:\n" + out)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
