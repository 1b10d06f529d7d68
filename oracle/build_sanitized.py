"""Builds and runs the oracle under the address and undefined-behaviour
sanitizers (CPU only, gcc; test infrastructure).

The driver ``san_driver.c`` calls every entry point of the oracle on small 2D
and 3D boxes of every boundary kind, gradient method and lattice, and the
configurations the oracle refuses; any invalid access, leak or undefined
operation aborts the run.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "_san", "san_driver")


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wno-unknown-pragmas",
           "-Wno-unused-function", "-I", HERE, os.path.join(HERE, "lbpf_oracle.c"),
           os.path.join(HERE, "san_driver.c"), "-o", EXE, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return EXE


def run() -> subprocess.CompletedProcess:
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    env.pop("LD_PRELOAD", None)
    return subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=600)


if __name__ == "__main__":
    build(verbose=True)
    r = run()
    print(r.stdout, r.stderr)
    sys.exit(r.returncode)
