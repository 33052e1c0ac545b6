"""Build-time check of the generated device code (runs on the build host only).

Compiles every HIP source of the library to device assembly and fails if any
instruction writes through the scalar data cache; the library uses vector
memory instructions for all its stores and atomics. Also checks that the
persistent batched step kernels keep a wave-uniform tile loop (no loop exit
taken lane by lane), which their termination relies on.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
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
    _check_uniform_tile_loops(asms)


# The exec-mask update that ends a loop for some lanes only.
_LANE_LOOP_EXIT = "s_andn2_b64 exec, exec"


def _loops_with_barrier_and_lane_exit(text):
    """(kernel, loop header) for every loop that holds a barrier and is left lane by lane.

    Uses the loop annotations the compiler writes on each block label
    ("This Loop Header", "in Loop: Header=...", "Parent Loop ...")."""
    out = []
    for m in re.finditer(r"^(_Z\w+):", text, re.M):
        end = text.find(".Lfunc_end", m.end())
        lines = text[m.end():end if end > 0 else len(text)].split("\n")
        cur, parent, members = None, {}, {}
        for n, line in enumerate(lines):
            lab = re.match(r"^(\.LBB(\w+)|; %bb\.\d+):", line)
            if lab:
                nxt = lines[n + 1] if n + 1 < len(lines) else ""
                both = line + nxt
                hm = re.search(r"Header=BB(\w+)", line)
                if "This Loop Header" in both or "This Inner Loop Header" in both:
                    cur = "BB" + lab.group(2) if lab.group(2) else cur
                    pm = re.search(r"Parent Loop BB(\w+)", both)
                    if pm and lab.group(2):
                        parent[cur] = "BB" + pm.group(1)
                elif hm:
                    cur = "BB" + hm.group(1)
                elif "in Loop" not in line:
                    cur = None
            if cur:
                members.setdefault(cur, []).append(n)
        has_barrier, lane_exit = set(), set()
        for h, idx in members.items():
            for n in idx:
                if "s_barrier" in lines[n]:
                    a = h
                    while a:
                        has_barrier.add(a)
                        a = parent.get(a)
                if _LANE_LOOP_EXIT in lines[n]:
                    lane_exit.add(h)
        out += [(m.group(1), h) for h in sorted(lane_exit & has_barrier)]
    return out


def _check_uniform_tile_loops(asms) -> None:
    """No loop that holds a barrier may be left lane by lane: a lane that left
    alone would park while the rest of its wave waited at the barrier, e.g.
    for a tile index that only the parked lane fetches (the persistent batched
    step kernel's tile loop)."""
    bad = []
    for a in asms:
        with open(a) as fh:
            bad += [f"{os.path.basename(a)}: {k} loop {h}" for k, h in _loops_with_barrier_and_lane_exit(fh.read())]
    if bad:
        raise RuntimeError("barrier inside a lane-divergent loop:\n" + "\n".join(bad[:20]))
