"""Build libqla.so (HIP, gfx950) in place, next to this file.

The translation units (host side, surrogate kernels, and the step kernel's
instances once per placement of the potentials and field triple) compile in
parallel, then link into one shared library.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
# (source, object name, defines)
SOURCES = [("qla.hip", "qla", ()), ("qnn.hip", "qnn", ())] + [
    ("qla_step_inst.hip", f"qla_step_m{m}_f{f}", (f"-DQLA_MODE={m}", f"-DQLA_FIELDS={f}"))
    for m in (0, 1) for f in (0, 1, 2)
]
LIB = os.path.join(HERE, "libqla.so")
INCLUDE = os.path.join(ROOT, "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay off (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def spilled_kernels(remarks: str) -> list:
    """Kernels that the compiler's resource-usage remarks show using scratch
    memory (register spills or a private array the compiler could not keep
    in registers): every kernel of the library is meant to need none, and
    one that does runs several times slower."""
    out, name = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and int(m.group(1)) > 0:
            out.append((name, int(m.group(1))))
    return out


def build(verbose: bool = False, extra=()) -> str:
    with tempfile.TemporaryDirectory(prefix="qla_build_") as tmpd:
        objs, procs = [], []
        for src, name, defs in SOURCES:
            obj = os.path.join(tmpd, name + ".o")
            cmd = [HIPCC, *FLAGS, *defs, *extra, "-Rpass-analysis=kernel-resource-usage", "-I", INCLUDE, "-I",
                   CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            # the remarks go to a file (a pipe could fill while the compiler runs)
            log = open(os.path.join(tmpd, name + ".log"), "w+")
            procs.append((name, subprocess.Popen(cmd, stderr=log), log))
            objs.append(obj)
        failed, spills = [], []
        for name, proc, log in procs:
            rc = proc.wait()
            log.seek(0)
            text = log.read()
            log.close()
            if rc != 0:
                failed.append(name)
                sys.stderr.write("\n".join(l for l in text.splitlines() if "remark:" not in l) + "\n")
            spills += spilled_kernels(text)
        if failed:
            raise RuntimeError(f"hipcc failed on {failed}")
        if spills:
            raise RuntimeError(f"kernels using scratch memory: {spills}")
        tmp = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
