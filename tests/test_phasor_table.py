"""The phasor table of the FP64 tile loops (gw_phasor_table.h) against its
generator: the committed header is what gen_phasor_table.py writes (table
entries rounded once from 60-digit values, remainder polynomials fitted in
60-digit arithmetic), and the scheme, evaluated operation by operation in
double as the kernels do, stays within 2e-16 of e^{-2 pi i x}."""
import os
import re
import subprocess
import sys

import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_1904_02863_amd", "csrc")


@pytest.fixture(scope="module")
def generated():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_phasor_table.py")], check=True,
                         capture_output=True, text=True).stdout
    return out


def test_header_is_the_generator_output(generated):
    with open(os.path.join(CSRC, "gw_phasor_table.h")) as fh:
        assert fh.read() == generated


def test_scheme_error(generated):
    m = re.search(r"worst absolute error .*: re ([0-9.e+-]+), im ([0-9.e+-]+)", generated)
    assert m is not None
    assert float(m.group(1)) < 2e-16 and float(m.group(2)) < 2e-16


def test_table_entries():
    import mpmath as mp
    with open(os.path.join(CSRC, "gw_phasor_table.h")) as fh:
        text = fh.read()
    n = int(re.search(r"#define GW_PHTAB_N (\d+)", text).group(1))
    rows = re.findall(r"\{(\S+), (\S+)\}", text)
    assert len(rows) == n == 2048
    mp.mp.dps = 40
    for k in (0, 1, 511, 512, 513, 1023, 1024, 1536, 2000, 2047):
        re_k, im_k = float.fromhex(rows[k][0]), float.fromhex(rows[k][1])
        assert re_k == float(mp.cospi(mp.mpf(2 * k) / n))
        assert im_k == float(-mp.sinpi(mp.mpf(2 * k) / n))
