"""Floating-point operations per point of the oracle's right-hand-side
expressions, counted by tracing the oracle's own C source
(tests/flops/oracle_flops.cpp): the method's operation count, stated beside
the count taken from the kernels' instruction stream.

The counter is pinned on the wave systems, whose counts follow by hand from
the 4th-order stencils written on neighbour differences:
  * second derivative: two differences and a sum per side pair (3 + 3), one
    weight, one subtraction, one division by 12 h^2 -> 9; the Laplacian is
    3 x 9 + 2 additions = 29, and du/dt = rho costs nothing;
  * first derivative: two differences, one weight, one subtraction, one
    division by 12 h -> 5; eq. (1) in first-order form needs d_i v_i
    (3 x 5 + 2) and d_i rho (3 x 5) -> 32."""
import json
import os
import shutil
import subprocess

import pytest

import bench

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def counter(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("flops") / "oracle_flops")
    subprocess.run([gxx, "-std=c++17", "-O1", "-fpermissive", "-w", "-o", exe,
                    os.path.join(HERE, "flops", "oracle_flops.cpp")], check=True)

    def run(*args):
        out = subprocess.run([exe, *map(str, args)], capture_output=True, text=True, check=True)
        return json.loads(out.stdout)
    return run


def test_counter_on_the_wave_systems(counter):
    w = counter("wave")
    assert w["raw"]["flops"] == w["cse"]["flops"] == 29
    assert w["cse"]["stencil"] == 29 and w["cse"]["div"] == 3
    w5 = counter("wave5")
    assert w5["raw"]["flops"] == w5["cse"]["flops"] == 32
    assert w5["cse"]["stencil"] == 32 and w5["cse"]["div"] == 6


def test_bssn_expression_count_matches_the_stated_figure(counter):
    b = counter("bssn", 4, 0, 1)
    print("BSSN 4th order, 1+log, Gamma-driver:", b)
    c = b["cse"]
    assert c["flops"] == bench.FLOPS_PER_POINT_EXPRESSION
    assert c["stencil"] + c["pointwise"] == c["flops"]
    assert b["raw"]["flops"] > c["flops"]  # the oracle recomputes; the expression does not
    # no transcendental function in the right-hand side
    assert all(c[k] == 0 for k in ("sqrt", "cbrt", "exp", "log", "pow", "sin", "cos"))


def test_higher_orders_cost_only_stencil_operations(counter):
    base = counter("bssn", 4, 0, 1)["cse"]
    for order in (6, 8):
        c = counter("bssn", order, 0, 1)["cse"]
        assert c["pointwise"] == base["pointwise"]
        assert c["stencil"] > base["stencil"]
