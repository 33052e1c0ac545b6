"""Build-time check of the generated device code (runs on the build host only).

Compiles every HIP source of the library to device assembly and fails if any
instruction writes through the scalar data cache; the library uses vector
memory instructions for all its stores and atomics.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

# Scalar-memory writes (stores, atomics, write-back of the scalar cache) are
# not used anywhere in this library; the device code is checked for them.
FORBIDDEN_PREFIXES = ("s_store", "s_atomic", "s_dcache_wb", "s_buffer_store", "s_scratch_store", "s_buffer_atomic")


def _device_asm(src: str, hipcc: str, flags, build_dir: str) -> str:
    out = os.path.join(build_dir, os.path.basename(src) + ".s")
    cmd = [hipcc, *flags, "--cuda-device-only", "-S", src, "-o", out]
    if src.endswith(".cpp"):
        cmd = [hipcc, *flags, "-x", "hip", "--cuda-device-only", "-S", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"device asm failed: {' '.join(cmd)}\n{r.stderr}")
    return out


def check_device_code(srcs, jobs, hipcc, flags, build_dir) -> None:
    """Fails if the device code of any source contains a scalar-memory write."""
    with cf.ThreadPoolExecutor(jobs) as ex:
        asms = list(ex.map(lambda s_: _device_asm(s_, hipcc, flags, build_dir), srcs))
    bad = []
    for a in asms:
        with open(a) as fh:
            for ln, line in enumerate(fh, 1):
                op = line.strip().split(" ", 1)[0]
                if op.startswith(FORBIDDEN_PREFIXES):
                    bad.append(f"{os.path.basename(a)}:{ln}: {line.strip()}")
    if bad:
        raise RuntimeError("scalar-memory writes in device code:\n" + "\n".join(bad[:20]))


