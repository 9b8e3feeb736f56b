"""Compile the C oracle (test infrastructure) into oracle/libsdpd_oracle.so
and, with OpenMP, into oracle/libsdpd_oracle_omp.so (the same source: its
parallel step variant then runs on several threads)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sdpd_oracle.c")
LIB = os.path.join(HERE, "libsdpd_oracle.so")
LIB_OMP = os.path.join(HERE, "libsdpd_oracle_omp.so")


def _compile(out: str, extra, verbose: bool):
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unknown-pragmas"] + extra + ["-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build_oracle(verbose: bool = False) -> str:
    """Compile with FP contraction off so that every product is rounded as
    written; -O2 only (no fast-math: the oracle must be IEEE-plain).  Both
    the single-threaded library and the OpenMP one."""
    _compile(LIB, [], verbose)
    _compile(LIB_OMP, ["-fopenmp"], verbose)
    return LIB


def _stale(lib: str) -> bool:
    return not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC)


def ensure_oracle() -> str:
    if _stale(LIB) or _stale(LIB_OMP):
        build_oracle()
    return LIB


def ensure_oracle_omp() -> str:
    ensure_oracle()
    return LIB_OMP


if __name__ == "__main__":
    print(build_oracle(verbose=True))
