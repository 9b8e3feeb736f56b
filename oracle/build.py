"""Compile the C oracle (test infrastructure) into oracle/libsdpd_oracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sdpd_oracle.c")
LIB = os.path.join(HERE, "libsdpd_oracle.so")


def build_oracle(verbose: bool = False) -> str:
    """Compile with FP contraction off so that every product is rounded as
    written; -O2 only (no fast-math: the oracle must be IEEE-plain)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_oracle() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build_oracle()
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))
