"""Host logic of the table role lock (Sec. 3.5 compatibility table), without a GPU: a C++ driver
runs the lock over a recording event backend from several threads and checks the recorded
dependency graph (every call ordered after every call of the group before it; calls of one group
on different streams left unordered)."""
import pathlib
import shutil
import subprocess

import pytest

SRC = pathlib.Path(__file__).parent / "cpp" / "roles_host_test.cpp"


@pytest.fixture(scope="module")
def binary(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = tmp_path_factory.mktemp("roles") / "roles_host_test"
    subprocess.run([gxx, "-O1", "-std=c++17", "-pthread", "-o", str(out), str(SRC)], check=True)
    return out


@pytest.mark.parametrize("mode", [1, 2], ids=["triple_group", "reader_writer"])
@pytest.mark.parametrize("threads,calls,seed", [(2, 500, 1), (8, 300, 2), (16, 100, 3)])
def test_role_lock_orders_groups(binary, mode, threads, calls, seed):
    r = subprocess.run([str(binary), str(mode), str(threads), str(calls), str(seed)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK")
    fields = r.stdout.split()
    shared = int(fields[fields.index("shared") + 2])
    assert shared > 0  # some groups held several calls at once
