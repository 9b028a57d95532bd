"""Instruction counts of the persistent kernel's trial-step loop.

Compiles the library source to gfx950 assembly with the build's flags
(`hipcc -S --cuda-device-only`) and, for each requested specialisation of
k_persistent<W, K0, K1, K2, RK>, counts the instructions in the basic blocks
of its innermost loop (the loop over trial steps between refill checks),
which is what one trial step of a wave issues.

    python -m paper_2304_02731_amd.loopcount 4,0,0,0,1 1,0,0,0,1 8,0,0,0,1
"""
from __future__ import annotations

import collections
import os
import re
import subprocess
import sys
import tempfile

from . import build as B


def assemble() -> str:
    """gfx950 assembly of qcams_api.hip, compiled with the library's flags."""
    flags = [f for f in B.FLAGS if f not in ("-fPIC", "-shared")]
    out = os.path.join(tempfile.mkdtemp(prefix="qcams_isa_"), "qcams_api.s")
    src = os.path.join(B.CSRC, "qcams_api.hip")
    subprocess.run([B.HIPCC] + flags + ["--cuda-device-only", "-S", "-o", out, src],
                   check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return open(out).read()


def _mangled(spec: str) -> str:
    """'4,0,0,0,1' -> the mangled template-argument prefix of k_persistent."""
    parts = []
    for v in (int(x) for x in spec.split(",")):
        parts.append("Li%sE" % (str(v) if v >= 0 else "n%d" % -v))
    return "_Z12k_persistentI" + "".join(parts) + "Ev"


def step_loop(asm: str, spec: str) -> list[str]:
    """Instructions of the innermost loop of k_persistent<spec> (the largest
    loop of depth 2, by the compiler's loop annotations)."""
    lines = asm.splitlines()
    head = _mangled(spec)
    start = [i for i, l in enumerate(lines) if l.startswith(head) and l.split(":")[0].endswith("Phl")]
    if not start:
        raise KeyError("no k_persistent<%s> in the assembly" % spec)
    body = []
    for l in lines[start[0]:]:
        if l.startswith(".Lfunc_end"):
            break
        body.append(l)
    best: list[str] = []
    for i, l in enumerate(body):
        if "Loop Header: Depth=2" not in l:
            continue
        m = re.match(r"^(\.LBB\w+):", body[i - 1])
        if not m:
            continue
        tag = "Header=" + m.group(1)[2:] + " "
        inloop, seq = False, []
        for j, x in enumerate(body):
            if re.match(r"^(\.LBB\w+:|; %bb)", x):
                inloop = (tag in x + " ") or j == i - 1
            elif inloop and x.startswith("\t") and not x.startswith(("\t.", "\t;")) and x.split():
                seq.append(x.strip())
        if len(seq) > len(best):
            best = seq
    return best


def main(argv: list[str]) -> int:
    specs = argv or ["4,0,0,0,1", "1,0,0,0,1", "8,0,0,0,1"]
    asm = assemble()
    for spec in specs:
        seq = step_loop(asm, spec)
        ops = collections.Counter(x.split()[0] for x in seq)
        valu = sum(v for k, v in ops.items() if k.startswith("v_"))
        f64 = sum(v for k, v in ops.items() if k.startswith("v_") and "f64" in k)
        print("k_persistent<%s>: %d instructions per trial step (%d vector, %d FP64 vector, "
              "%d scalar loads)" % (spec, len(seq), valu, f64,
                                    sum(v for k, v in ops.items() if k.startswith("s_load"))))
        print("  " + ", ".join("%s %d" % kv for kv in ops.most_common(12)))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
