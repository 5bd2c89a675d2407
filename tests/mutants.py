"""Planted mistakes in the CPU oracle, for checking that a pin can fail.

``mutant(old, new, count)`` compiles a copy of the oracle's C source with the
text ``old`` replaced by ``new`` (it must occur exactly ``count`` times) into
a temporary library, and points the ``oracle`` package at it for the
duration of the ``with`` block.  The oracle's own source and library are
never touched.
"""
import contextlib
import os
import subprocess
import tempfile

import oracle


@contextlib.contextmanager
def mutant(old: str, new: str, count: int = 1):
    src = open(oracle._SRC).read()
    found = src.count(old)
    assert found == count, f"planted mistake: {old!r} found {found} times, expected {count}"
    with tempfile.TemporaryDirectory() as d:
        # the oracle includes its own header: compile the copy next to it
        c_path = os.path.join(d, "raytrace_oracle_mutant.c")
        with open(c_path, "w") as f:
            f.write(src.replace(old, new))
        lib = os.path.join(d, "liboracle_mutant.so")
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                        "-shared", "-fPIC", "-I", os.path.dirname(oracle._SRC), "-o", lib,
                        c_path, "-lm", "-lpthread"], check=True)
        saved = oracle._LIB, oracle._lib
        oracle._LIB, oracle._lib = lib, None
        try:
            yield oracle
        finally:
            oracle._LIB, oracle._lib = saved
