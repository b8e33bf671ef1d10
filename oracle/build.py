"""Build step for the oracle library (plain C, gcc).  Test infrastructure."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False, src: str | None = None, out: str | None = None) -> str:
    """Compile the oracle (or, for the pin-strength tests, a modified copy of
    its source `src` into `out`)."""
    out = out or os.path.join(HERE, "libsccg_oracle.so")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-ffp-contract=off", "-I", HERE,
           src or os.path.join(HERE, "sccg_oracle.c"), "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
