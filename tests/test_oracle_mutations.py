"""The oracle's pins have teeth: each deliberately broken copy of oracle.c
(a wrong sign, an open ball, a dropped term, transposed indexing, a strict
merge, kept zero-length pieces, a different border rule) is compiled on the
CPU and must fail the pin suite."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "chord_sign": ("round_end(z[2 * i] - h, mode)", "round_end(z[2 * i] + h, mode)"),
    "open_ball": ("if (d2 <= r2) {", "if (d2 < r2) {"),
    "dropped_d2": ("double h = sqrt(r2 - d2);", "double h = sqrt(r2);"),
    "transposed_index": ("int64_t cc = (int64_t)yy * nx + xx;", "int64_t cc = (int64_t)xx * ny + yy;"),
    "strict_merge": ("if (v[i].lo <= v[m].hi) {", "if (v[i].lo < v[m].hi) {"),
    "keep_zero_length": ("if (hi > lo) {", "if (hi >= lo) {"),
    "border_empty": ("if (xx < 0 || xx >= nx || yy < 0 || yy >= ny) continue;",
                     "if (xx < 0 || xx >= nx || yy < 0 || yy >= ny) { if (op == ORACLE_ERODE) ivec_push(&cand, -INFINITY, INFINITY); continue; }"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(tmp_path, name):
    sys.path.insert(0, ROOT)
    import oracle
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    oracle.compile_source(str(mut), str(lib))
    env = dict(os.environ, ORACLE_LIB=str(lib))
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, f"mutant {name} passed every pin:\n{res.stdout[-2000:]}"
