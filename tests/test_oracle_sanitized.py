"""The oracle under the address and undefined-behaviour sanitizers (CPU only).

A gcc build of ``oracle/lbpf_oracle.c`` with ``-fsanitize=address,undefined``
runs ``oracle/san_driver.c``, which calls every oracle entry point on small
boxes of every boundary kind, gradient method, lattice and anisotropy kind,
and the configurations the oracle refuses.  Any invalid access, leak or
undefined operation ends the run with a sanitizer report.
"""
import os
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_sanitizers():
    from oracle import build_sanitized as B
    B.build()
    r = B.run()
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out
    assert "all checks passed" in r.stdout
