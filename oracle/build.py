"""Build the FP64 CPU oracle (test infrastructure only) into oracle/libcg_oracle.so.

Plain gcc, -O2, no fused multiply-add contraction and no fast-math, so the oracle's
arithmetic is the literal IEEE double sequence written in cg_oracle.c; OpenMP for the
optional parallel per-node loops (off unless a thread count is set).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cg_oracle.c")
LIB = os.path.join(HERE, "libcg_oracle.so")


def build(sanitize: bool = False, out: str = None) -> str:
    out = out or (os.path.join(HERE, "libcg_oracle_san.so") if sanitize else LIB)
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", SRC, "-o", out, "-lm"]
    if sanitize:
        cmd[3:3] = ["-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    else:  # per-node loops in parallel when asked for (ora_set_threads); same results
        cmd[3:3] = ["-fopenmp"]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(sanitize="--sanitize" in sys.argv))
