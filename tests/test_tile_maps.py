"""The transpose tile's index maps on the host (no GPU): exact cover of the
LDS tile and of the dst tile, the swizzle undone on every read, the barrier
placement (required exactly where LDS ownership changes hands, Section 3.3)
and conflict-free LDS reads under a 64-bank model, for every tile geometry
the kernels instantiate (tests/native/tile_map_check.cpp over the kernels' own
tile_map.h).  Planted mistakes in a copy of the header must be caught."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CHECK = os.path.join(HERE, "native", "tile_map_check.cpp")
HEADER = os.path.join(ROOT, "paper_2605_13864_amd", "csrc", "tile_map.h")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def run_check(tmp_path, header=HEADER):
    exe = os.path.join(tmp_path, "tile_map_check")
    subprocess.run(["g++", "-std=c++17", "-O1", f'-DTILE_MAP_H="{header}"', "-o", exe, CHECK],
                   check=True)
    return subprocess.run([exe], capture_output=True, text=True)


def test_tile_maps(tmp_path):
    r = run_check(tmp_path)
    assert r.returncode == 0 and "all tile maps ok" in r.stdout, r.stdout[-3000:]
    assert r.stdout.count("ok=1") == 37


MUTANTS = [
    ("swizzle_off", "return k ^ (((row / V) ^ ((row % V) * (16 / V))) & 15);", "return k;"),
    ("swizzle_row_only", "return k ^ (((row / V) ^ ((row % V) * (16 / V))) & 15);",
     "return k ^ ((row / V) & 15);"),
    ("phase1_rows_strided_wrong", "static constexpr int p1_row(int t, int p) { return t / P + RP * p; }",
     "static constexpr int p1_row(int t, int p) { return t / P + RP * p + (p & 1); }"),
    ("phase2_row_of_wrong_piece", "return (k * EPW + e) * SC + swz<EB>(k * EPW + e, m);",
     "return (k * EPW + e) * SC + swz<EB>(k * EPW, m);"),
    ("lds_rows_overlap", "return (row * SC + swz<EB>(row, byte >> 4)) * 16 + (byte & 15);",
     "return ((row * SC - (row & 1)) + swz<EB>(row, byte >> 4)) * 16 + (byte & 15);"),
]


@pytest.mark.parametrize("name,orig,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_tile_map_mutants_caught(tmp_path, name, orig, bad):
    src = open(HEADER).read()
    assert src.count(orig) == 1, name
    h = os.path.join(tmp_path, "tile_map.h")
    with open(h, "w") as f:
        f.write(src.replace(orig, bad))
    r = run_check(tmp_path, h)
    assert r.returncode != 0, f"mutant {name} not caught:\n{r.stdout[-2000:]}"
