"""Build step of the HIP library: hipcc for gfx950 into libmicx.so (in-tree)."""
from __future__ import annotations

import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmicx.so")
SOURCES = ["micx_api.hip", "micx_kernels.hip", "micx_dp.hip", "micx_noalloc.hip", "micx_dp_co.hip"] + [
    "micx_dp_%s_%s%d.hip" % (v, f, k) for f in ("i", "g") for v in ("f64", "u32") for k in range(5)]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags():
    return [
        "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed FP32 instructions stay off: plain FP32 code only
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        "-I" + INCLUDE, "-I" + CSRC,
    ]


# Extra flags per source.  The DP takes minima of finite values only, so it is
# compiled without NaN semantics (v_min_f64 needs no operand canonicalisation).
EXTRA = {s: ["-fno-honor-nans"] for s in SOURCES if s.startswith("micx_dp")}


# The DP kernels must not spill: their resource usage is read back from the
# compiler and the build fails if any of them uses private (scratch) memory or
# accumulation registers (AGPRs, where the compiler parks VGPRs it cannot fit;
# such spills also push a kernel past its occupancy step).
USAGE_FLAG = "-Rpass-analysis=kernel-resource-usage"
_DP_NAME = re.compile(r"k_dpI([dj])Li(\d+)ELi(\d+)ELi(\d+)E")


def dp_resource_usage(text):
    """Parse the compiler's kernel-resource-usage remarks: {(fx, NL, YR, T):
    {"VGPRs": .., "AGPRs": .., "ScratchSize": .., ...}} for the DP kernels."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            k = _DP_NAME.search(m.group(1))
            cur = (int(k.group(1) == "j"), int(k.group(2)), int(k.group(3)), int(k.group(4))) if k else None
            if cur is not None:
                out[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[bytes/lane\])?: (\d+)", line)
        if m and cur is not None:
            out[cur][m.group(1).strip()] = int(m.group(2))
    return out


def spilling(usage):
    """DP instances (fx, NL, YR, T) whose resource usage shows a spill:
    scratch memory, spilled VGPRs or accumulation registers."""
    return sorted(k for k, u in usage.items()
                  if u.get("ScratchSize", 0) or u.get("VGPRs Spill", 0) or u.get("AGPRs", 0))


def _compile(src, obj, verbose, defines=(), check_spills=True, device_only=False):
    dp = src.startswith("micx_dp_")
    cmd = [HIPCC] + flags() + EXTRA.get(src, []) + list(defines) + ([USAGE_FLAG] if dp else [])
    cmd += (["--cuda-device-only"] if device_only else []) + ["-c", "-o", obj, os.path.join(CSRC, src)]
    cmd = [c for c in cmd if c != "-shared"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s%s" % (src, res.stdout, res.stderr))
    usage = dp_resource_usage(res.stderr) if dp else {}
    if check_spills:
        bad = spilling(usage)
        if bad:
            raise RuntimeError("DP kernels of %s spill registers (fx, NL, YR, T): %s" % (src, bad))
    return usage


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every HIP source (in parallel) and link paper_1208_4271_amd/libmicx.so
    (or `out`; `defines` are extra -D flags for the build-time tuning knobs)."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(os.path.dirname(os.path.abspath(out)), "_build",
                          os.path.basename(out).replace(".so", ""))
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES]
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose, defines), zip(SOURCES, objs)))
    LIBOUT = out
    tmp = LIBOUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIBOUT)
    return LIBOUT


CALIB_SRC = os.path.join(HERE, "calib", "valu_rate.hip")
CALIB_BIN = os.path.join(HERE, "calib", "valu_rate")


def build_calib(verbose: bool = False) -> str:
    """Compile the VALU issue-rate program (a standalone executable)."""
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-O3", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-o", CALIB_BIN, CALIB_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s%s" % (CALIB_SRC, res.stdout, res.stderr))
    return CALIB_BIN


if __name__ == "__main__":
    print(build(verbose=True))
