"""The algorithmic flop counts the benchmark's roofline uses are the
oracle's own operation counts: its C source compiled with a counting scalar
type (tests/opcount/counted_oracle.cpp; an operation with a state-dependent
operand is one flop, operations on material and grid constants are not
counted), per interior cell of large periodic boxes."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def counts(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("opcount") / "counted_oracle")
    subprocess.run(["g++", "-std=c++17", "-O2", "-fpermissive", "-w", "-o", exe,
                    os.path.join(HERE, "opcount", "counted_oracle.cpp"), "-lm"], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return json.loads(out)


def test_building_blocks(counts):
    # fixed by the formulation: primitive recovery, the SSP-RK3 combinations
    # q0 + dt L, 3/4 q0 + 1/4 (q + dt L), 1/3 q0 + 2/3 (q + dt L)
    assert counts["cons_to_prim_3d"] == 28
    assert counts["rk3_stage"] == [2, 5, 5]
    assert counts["weno5_pair"] == 99
    assert 140 <= counts["hllc_face"] <= 170


def test_bench_flop_constants_are_the_counted_ones(counts):
    import bench
    rk3 = sum(counts["rk3_stage"]) / 3
    total3 = counts["rhs_per_cell_3d"] + 7 * rk3
    assert bench.FLOPS_PER_CELL_UPDATE == pytest.approx(total3, rel=2e-3)
    # per direction: (rhs - primitive recovery - the div(u) source) / 3; the
    # x+y kernel does two directions and forms the stage combination
    per_dir = (counts["rhs_per_cell_3d"] - counts["cons_to_prim_3d"] - 2) / 3
    assert bench.SPLIT[0]["flops"] == pytest.approx(counts["cons_to_prim_3d"] + 2 * per_dir + 7 * rk3, rel=2e-3)
    assert bench.SPLIT[0]["flops"] + bench.SPLIT[1]["flops"] == bench.FLOPS_PER_CELL_UPDATE
    total2 = counts["rhs_per_cell_2d"] + 6 * rk3
    assert bench.FLOPS_PER_CELL_UPDATE_2D == pytest.approx(total2, rel=2e-3)
