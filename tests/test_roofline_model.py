"""The flop/byte model reproduces Table 1 (Sec. 1) as printed."""
import os

import pytest

from paper_1411_4439_amd import roofline as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_flop_per_byte.txt")


def _table1():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, full, r14 = line.split()
                rows.append((int(n), float(full), float(r14)))
    return rows


def test_table1_reproduced_to_two_decimals():
    rows = _table1()
    assert len(rows) == 7
    for n, full, r14 in rows:
        assert round(R.paper_flop_per_byte(n, "full"), 2) == pytest.approx(full, abs=1e-9), n
        assert round(R.paper_flop_per_byte(n, "r14"), 2) == pytest.approx(r14, abs=1e-9), n


def test_double_precision_halves_intensity():
    for n in (1, 4, 8):
        assert R.paper_flop_per_byte(n, "full", "f64") == pytest.approx(R.paper_flop_per_byte(n, "full") / 2)


def test_four_over_one_rhs_gain():
    # the CG gain of 4 rhs over 1 rhs is compared with the r14 Dslash intensity ratio, 2.16
    assert round(R.paper_flop_per_byte(4, "r14") / R.paper_flop_per_byte(1, "r14"), 2) == 2.16


def test_algorithmic_bytes():
    assert R.dslash_algorithmic_bytes_per_site(8) == 1152 + 48 * 8
    assert R.dslash_algorithmic_bytes_per_site(8, "r14") == 1024 + 48 * 8
    assert R.dslash_algorithmic_bytes_per_site(1, "full", "f64") == 2304 + 96
    assert R.cg_iteration_bytes_per_site(8) == 2304 + 264 * 8
