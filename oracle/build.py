"""Compile the CPU oracle (test infrastructure) with gcc.

Two shared objects are produced next to this file:
  liboracle.so      double precision (the oracle proper)
  liboracle_f32.so  the same source in single precision (precision-floor probe)
Built at -O2 without -ffast-math so the arithmetic follows the source order.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB64 = os.path.join(HERE, "liboracle.so")
LIB32 = os.path.join(HERE, "liboracle_f32.so")


def build(force=True):
    for out, extra in ((LIB64, []), (LIB32, ["-DORACLE_FLOAT"])):
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-fno-fast-math", "-ffp-contract=off", *extra, SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return LIB64, LIB32


if __name__ == "__main__":
    print(build())
