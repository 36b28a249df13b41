"""Host-side checks of bench.py (no GPU): the one-GPU contract, the algorithmic byte models on
cases whose value follows from their definitions, and the measured-traffic records, which are
reported only for the sources they were taken on."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2603_17168_amd import cskv  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, cwd=ROOT, capture_output=True,
                       text=True, env={**os.environ, **env}, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_find_byte_model():
    V = 4 * 32
    # a miss reads the key, both digest lines and its false-positive key granules, writes the flag
    assert bench.find_bytes_per_key(32, 0.0, 1.0, 0.0) == 8 + 2 * 128 + 1 + 64
    # a hit in b1: key, digest line, one key granule, the row read and written, the flag
    assert bench.find_bytes_per_key(32, 1.0, 0.5, 0.0) == 8 + 128 + 64 + 2 * V + 1
    # a hit in b2 adds b2's digest line and b1's false positives (half a granule per full line)
    assert bench.find_bytes_per_key(32, 1.0, 1.0, 1.0) == 8 + 128 + 64 + 2 * V + 1 + 128 + 0.5 * 64
    # linear in the hit rate
    lo, hi = bench.find_bytes_per_key(32, 0.0, 0.7, 0.4), bench.find_bytes_per_key(32, 1.0, 0.7, 0.4)
    assert bench.find_bytes_per_key(32, 0.5, 0.7, 0.4) == pytest.approx((lo + hi) / 2)


def test_upsert_byte_models():
    V = 4 * 32
    insert = 8 + V + 2 * 128 + 0.5 * 64 + 3 * 64 + V + 1
    assert bench.upsert_bytes_contract(32, 0.5, {cskv.ST_INSERTED: 10}) == pytest.approx(insert)
    evict = insert + 2 * 8 * 128 + 64
    mixed = bench.upsert_bytes_contract(32, 0.5, {cskv.ST_INSERTED: 1, cskv.ST_INSERTED_EVICT: 3})
    assert mixed == pytest.approx((insert + 3 * evict) / 4)
    # the priced model: phase D2 reads the candidates' minima (a granule each) per key, and the
    # score and key lines (16 lines) once per touched bucket, shared by that bucket's keys
    assert bench.upsert_bytes_model(32, 0.5, {cskv.ST_INSERTED: 7}, 1 << 20, 1 << 19) == pytest.approx(insert)
    share = 16 * 128 * (1 << 19) * (1 - np.exp(-2.0)) / (1 << 20)
    assert bench.upsert_bytes_model(32, 1.0, {cskv.ST_INSERTED_EVICT: 5}, 1 << 20, 1 << 19) == pytest.approx(
        8 + V + 2 * 128 + 64 + 3 * 64 + V + 1 + 3 * 64 + share)
    assert bench.upsert_bytes_model(32, 1.0, {cskv.ST_REJECTED: 5}, 1 << 20, 1 << 19) == pytest.approx(
        8 + 2 * 128 + 2 * 64 + 64 + 1 + share)


def test_traffic_records_follow_their_sources(monkeypatch):
    loads = [0.5, 0.75, 0.9, 1.0]
    batch = 1 << 20
    # a record taken on the sources as they are now is reported: the mean over the bench's launches
    monkeypatch.setitem(bench.FIND_TRAFFIC, "source_sha256", bench.source_sha256(bench.FIND_SOURCES))
    monkeypatch.setitem(bench.UPSERT_TRAFFIC, "source_sha256", bench.source_sha256(bench.UPSERT_SOURCES))
    per = bench.FIND_TRAFFIC["per_key"]
    want = sum(per[f"{x:.2f}"]["hit100"] + per[f"{x:.2f}"]["hit50"] for x in loads) * batch / (2 * len(loads))
    assert bench.find_traffic_per_launch(32, loads, batch) == pytest.approx(want)
    up = bench.UPSERT_TRAFFIC["per_key"]
    want_u = sum(up[f"{x:.2f}"] for x in loads) * batch / len(loads)
    assert bench.upsert_traffic_per_launch(32, loads, batch) == pytest.approx(want_u)
    # another dim, a load without a record, or changed sources give no figure
    assert bench.find_traffic_per_launch(64, loads, batch) is None
    assert bench.upsert_traffic_per_launch(32, [0.6], batch) is None
    monkeypatch.setitem(bench.FIND_TRAFFIC, "source_sha256", "0" * 64)
    monkeypatch.setitem(bench.UPSERT_TRAFFIC, "source_sha256", "0" * 64)
    assert bench.find_traffic_per_launch(32, loads, batch) is None
    assert bench.upsert_traffic_per_launch(32, loads, batch) is None


def test_source_hashes_are_stable_and_distinct():
    h1 = bench.source_sha256(bench.UPSERT_SOURCES)
    assert h1 == bench.source_sha256(bench.UPSERT_SOURCES)
    assert h1 != bench.source_sha256(bench.FIND_SOURCES)
    assert len(h1) == 64
