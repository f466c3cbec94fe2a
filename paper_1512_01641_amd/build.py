"""Build libnwmine.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1512_01641_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnwmine.so")
SOURCES = ["k_expand.hip", "k_score.hip", "k_align.hip", "k_backward.hip", "k_bidir.hip", "nwm_abi.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # FP32 DP must be bit-exact: no contraction into FMA, IEEE denormals
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    # no packed-FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    # MFMA accumulators in ordinary VGPRs: no accumulator copies between the
    # unrolled K chunks of the contraction
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


# Kernels whose memory waits are explicit counts over a fixed sequence of
# memory operations (inline asm loads the compiler does not track): a spill
# to scratch would add memory operations and silently shift those counts, so
# the build fails if any of them uses scratch.
NO_SCRATCH = {"k_align.hip": ("k_nw_fill", "k_nw_walk")}


def resource_usage(text: str) -> dict:
    """Per-kernel {'ScratchSize', 'VGPRs', ...} from the compiler's
    kernel-resource-usage remarks (mangled kernel name -> fields)."""
    out, cur = {}, None
    for line in text.splitlines():
        if "remark:" not in line:
            continue
        body = line.split("remark:", 1)[1].split("[-Rpass", 1)[0].strip()
        if body.startswith("Function Name:"):
            cur = body.split(":", 1)[1].strip()
            out[cur] = {}
        elif cur is not None and ":" in body:
            k, v = body.rsplit(":", 1)
            try:
                out[cur][k.strip()] = int(v.strip())
            except ValueError:
                pass
    return out


def check_scratch(src: str, text: str) -> None:
    guarded = NO_SCRATCH.get(src, ())
    if not guarded:
        return
    usage = resource_usage(text)
    seen = set()
    for name, fields in usage.items():
        for g in guarded:
            if g in name:
                seen.add(g)
                if fields.get("ScratchSize [bytes/lane]", 0) != 0:
                    raise RuntimeError("%s: kernel %s uses scratch (%d bytes/lane); its explicit memory waits "
                                       "assume no spills" % (src, name, fields["ScratchSize [bytes/lane]"]))
    missing = set(guarded) - seen
    if missing:
        raise RuntimeError("%s: no resource-usage remarks for %s" % (src, sorted(missing)))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    remarks = ["-Rpass-analysis=kernel-resource-usage"] if src in NO_SCRATCH else []
    cmd = [HIPCC, *FLAGS, *remarks, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    check_scratch(src, r.stdout + r.stderr)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
