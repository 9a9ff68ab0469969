"""Build libpermhip.so (HIP, gfx950) in-tree.

Every translation unit is compiled with hipcc in parallel into
paper_1606_05836_amd/_build/, then linked into paper_1606_05836_amd/libpermhip.so.
The size-range kernel file is compiled once per range.  The kernel resource
report is checked: a sweep kernel that spills registers is a build error
(the sweep keeps update columns resident in VGPRs and reads them with DPP
row broadcasts, which is only safe when no spill code rewrites them).

usage: python -m paper_1606_05836_amd.build [--jobs N]
"""
from __future__ import annotations

import argparse
import hashlib
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpermhip.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", CSRC, "-I", os.path.join(ROOT, "include"),
    "-Rpass-analysis=kernel-resource-usage",
]

DPP_NMAX = 44  # keep equal to DPP_NMAX in csrc/sweep.hpp
BATCHED_DPP_NMAX = 40  # keep equal to BATCHED_DPP_NMAX in csrc/sweep_batched.hip
RANGES = [(1, 16), (17, 24), (25, 32), (33, 40), (41, 44), (45, 52)]
RANGED = ("sweep_single.hip", "sweep_batched.hip")  # compiled once per size range


def build_id() -> str:
    """Hash of the kernel and header sources: the autotuner's cache entries
    are valid for one build id only."""
    h = hashlib.sha256()
    for d in (CSRC, os.path.join(ROOT, "include")):
        for name in sorted(os.listdir(d)):
            if name.endswith((".hip", ".cpp", ".hpp", ".h")):
                with open(os.path.join(d, name), "rb") as f:
                    h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def units():
    """(output object, source, extra flags)"""
    u = []
    for lo, hi in RANGES:
        for src in RANGED:
            u.append((f"{src[:-4]}_{lo}_{hi}.o", src, [f"-DPH_NLO={lo}", f"-DPH_NHI={hi}"]))
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp")) and name not in RANGED:
            u.append((os.path.splitext(name)[0] + ".o", name, []))
    return u


_REMARK = re.compile(r"remark: .*?(Function Name|VGPRs Spill|SGPRs Spill|AGPRs|VGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]): (\S+)")


def _compile(unit):
    obj, src, extra = unit
    cmd = [HIPCC, *FLAGS, f'-DPH_BUILD_ID="{build_id()}"', *extra, "-c", os.path.join(CSRC, src),
           "-o", os.path.join(OUT, obj)]
    p = subprocess.run(cmd, capture_output=True, text=True)
    return unit, p.returncode, p.stdout + p.stderr


def _resources(log: str):
    """kernel name -> dict of the resource remarks."""
    res, cur = {}, None
    for m in _REMARK.finditer(log):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = val
            res[cur] = {}
        elif cur is not None:
            res[cur][key] = val
    return res


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    us = units()
    # biggest kernels first so the long compiles start early
    us.sort(key=lambda u: -int(u[2][1].split("=")[1]) if u[2] else 0)
    errors, report = [], {}
    with ThreadPoolExecutor(jobs) as ex:
        for (obj, src, extra), rc, log in ex.map(_compile, us):
            if rc != 0:
                errors.append(f"{src} {' '.join(extra)}:\n" + "\n".join(
                    l for l in log.splitlines() if "remark:" not in l)[-4000:])
            report.update(_resources(log))
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n\n".join(errors))
    with open(os.path.join(OUT, "resources.txt"), "w") as f:
        for k in sorted(report):
            f.write(k + " " + " ".join(f"{a}={b}" for a, b in sorted(report[k].items())) + "\n")
    def _uses_dpp(kernel):
        if "k_minors" in kernel:  # csrc/minors.hip keeps resident columns too
            return True
        if "k_gradILi" in kernel:  # csrc/grad.hip: DPP and lane-swap exchanges every term
            return True
        if "k_ryser_paired_2l" in kernel:  # csrc/ryser_paired.hip: resident columns of the two-lane walk
            return True
        m = re.search(r"sweep_\w*?ILi(\d+)E(Li(\d+)E)?", kernel)
        if not m:
            return False
        # batched kernels are templated on the bucket bounds: DPP is used
        # there when the bucket starts at or below BATCHED_DPP_NMAX
        if "batched" in kernel:
            return int(m.group(1)) <= BATCHED_DPP_NMAX
        # one-matrix sweeps: one lane per term up to n = 48 (resident columns
        # up to DPP_NMAX, a staged column in the same layout from n = 24),
        # two lanes per term from PAIR_NMIN on (csrc/ph_internal.hpp); all
        # read update columns with DPP
        return True

    # kernels that read resident columns with DPP: no spill code of any kind
    # (AGPR copies included) is allowed there, and no per-lane array may have
    # been left in scratch memory (a register array the compiler could not
    # keep in registers, e.g. one indexed through a merged pointer)
    bad = [k for k, v in report.items() if ("sweep" in k or "k_minors" in k or "k_gradILi" in k
                                             or "k_ryser_paired_2l" in k) and _uses_dpp(k) and (
        v.get("VGPRs Spill", "0") != "0" or v.get("SGPRs Spill", "0") != "0" or v.get("AGPRs", "0") != "0"
        or v.get("ScratchSize [bytes/lane]", "0") != "0")]
    if bad:
        raise RuntimeError("sweep kernels spill registers or use scratch: " + ", ".join(bad[:8]))
    objs = [os.path.join(OUT, u[0]) for u in us]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-ldl"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(objs)} objects")
    return LIB


def clean():
    shutil.rmtree(OUT, ignore_errors=True)
    if os.path.exists(LIB):
        os.remove(LIB)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--clean", action="store_true")
    a = ap.parse_args()
    if a.clean:
        clean()
    build(a.jobs, verbose=True)
    sys.exit(0)
