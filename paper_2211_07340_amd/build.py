"""Build the HIP library ``libsdtw.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsdtw.so")
SOURCES = ["api.hip", "prep.hip", "align.hip", "scores.hip", "wide.hip", "events.hip"]
ARCH = os.environ.get("SDTW_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # exact IEEE arithmetic: no contraction, no fast-math, fp32 denormals kept
    "-ffp-contract=off", "-fno-fast-math",
    # no packed-fp32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


PROBE_LIB = os.path.join(HERE, "libsdtw_probe.so")
PROBE_SOURCES = ["probe_issue.hip"]


def build_probe(verbose: bool = False) -> str:
    """The VALU issue-rate probe (libsdtw_probe.so, measurement tooling)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *FLAGS, "-o", PROBE_LIB + ".tmp",
           *[os.path.join(CSRC, s) for s in PROBE_SOURCES]]
    proc = subprocess.run(cmd, capture_output=True, text=True, cwd=HERE)
    out = "\n".join(l for l in (proc.stdout + proc.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed ({proc.returncode}):\n{out}")
    if verbose and out.strip():
        print(out, file=sys.stderr)
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    return PROBE_LIB


def build(verbose: bool = False, save_temps: str | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *FLAGS, "-o", LIB + ".tmp", *[os.path.join(CSRC, s) for s in SOURCES]]
    if save_temps:
        os.makedirs(save_temps, exist_ok=True)
        cmd.insert(1, f"-save-temps={'obj'}")
    proc = subprocess.run(cmd, capture_output=True, text=True, cwd=save_temps or HERE)
    out = "\n".join(l for l in (proc.stdout + proc.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if proc.returncode != 0:
        raise RuntimeError(f"hipcc failed ({proc.returncode}):\n{out}")
    if verbose and out.strip():
        print(out, file=sys.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_probe(verbose=True))
