"""Build and run the streaming-bandwidth probe (csrc/stream_probe.hip), the
yardstick for the vertex step's measured HBM traffic rate.  A standalone HIP
program; it uses nothing from the library.

    python -m paper_2102_12933_amd.stream_probe          # build if needed, run
"""
from __future__ import annotations

import os
import subprocess
import sys

from paper_2102_12933_amd.build import ARCH, DEVICE_FLAGS, HIPCC

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "stream_probe.hip")
EXE = os.path.join(HERE, "stream_probe")


def build() -> str:
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", *DEVICE_FLAGS, SRC, "-o", EXE + ".tmp"]
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(EXE + ".tmp", EXE)
    return EXE


def main() -> int:
    if not os.path.exists(EXE):
        build()
    return subprocess.run([EXE]).returncode


if __name__ == "__main__":
    sys.exit(main())
