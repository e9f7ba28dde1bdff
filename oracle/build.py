"""Build the CPU oracle library (test infrastructure only).

Compiles ``haf_oracle.c`` with the host C compiler into ``oracle/_build/liboracle.so``.
Plain IEEE double / long double arithmetic: no fast-math, no FMA contraction.
"""
import os
import pathlib
import subprocess
import sys

HERE = pathlib.Path(__file__).resolve().parent
SRC = HERE / "haf_oracle.c"
OUT = HERE / "_build" / "liboracle.so"

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fcx-limited-range"]


def build(force: bool = False) -> pathlib.Path:
    OUT.parent.mkdir(parents=True, exist_ok=True)
    if not force and OUT.exists() and OUT.stat().st_mtime >= SRC.stat().st_mtime:
        return OUT
    cc = os.environ.get("CC", "gcc")
    tmp = OUT.with_suffix(".so.tmp%d" % os.getpid())
    subprocess.run([cc, *CFLAGS, "-o", str(tmp), str(SRC), "-lm"], check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
