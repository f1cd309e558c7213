"""The integer constructions of the multimodular residue split (nearest quotient from one
fused multiply-add against 1.5 2^52, or 1.5 2^23 in single precision; residue modulo 2^24
from one 24-bit multiply-add), run on the CPU with IEEE fma and checked against residues
from integer division, for every modulus of the moduli set (Strategy 3 of Section 6.1:
balanced residues modulo the small moduli)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_residue_constructions_match_integer_division(tmp_path):
    exe = tmp_path / "residue_arith_check"
    subprocess.run(["gcc", "-O2", "-std=c99", "-o", str(exe), os.path.join(HERE, "residue_arith_check.c"), "-lm"],
                   check=True)
    out = subprocess.run([str(exe), "200000"], check=True, capture_output=True, text=True, timeout=300).stdout
    assert out.startswith("ok "), out
    assert int(out.split()[1]) > 16 * 200000
