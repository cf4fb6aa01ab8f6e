"""The task graph of the persistent diagonal-block factorisation
(csrc/dag.hpp), emulated on the CPU (tests/native/dag_emulate.cpp, built with
g++) through the launch's protocol -- workers take tasks in list order and
wait on readiness counters -- with 1 to 512 workers and random completion
orders, in the chained form the launches use (the tile-to-tile chain as one
task that publishes its solve midway) and the unchained one: the list only
waits on earlier tasks, the workers never deadlock,
tasks runnable together never conflict on a tile, and the tasks, executed
as plain dense tile operations, give L^{-1} and log|A| of a random SPD
matrix against a plain Cholesky and triangular inversion -- for 1 to 43
tiles and several blocks per launch."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_dag_task_lists_emulated(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "dag_emulate")
    src = os.path.join(HERE, "native", "dag_emulate.cpp")
    subprocess.run([gxx, "-O2", "-std=c++17", src, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count("ok chained") == 7 * 5 + 2 * 3
    assert r.stdout.count("ok unchained") == 7 * 5 + 2 * 3
