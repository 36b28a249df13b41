"""GPU parity of route sub-rounds (a semantic setting: an upsert call's distinct keys, ordered by
last occurrence, routed and applied in r chunks, each against the table the chunks before it
left): every call against the oracle with the same setting, bit for bit, with duplicates,
reserved keys, evictions and find_or_insert; programs built with the setting (serial and
overlapped, eager and captured) against plain calls; stale programs refuse to launch."""
import sys

import numpy as np
import pytest
import torch

from paper_2603_17168_amd import cskv
from paper_2603_17168_amd.workload import as_u64, batch_schedule, keys as gen_keys, program_inputs
from tests.parity import Twin
from tests.test_gpu_program import build_program, fresh_outputs, prefilled, run_calls, same_outputs, same_tables

pytestmark = pytest.mark.gpu
M64 = (1 << 64) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def np_keys(stream, n, start=0):
    return as_u64(gen_keys(stream, n, start))


@pytest.mark.parametrize("r", [2, 3, 17, 64])
@pytest.mark.parametrize("mode,policy", [("dual", "custom"), ("dual", "lru"), ("single", "lfu")])
def test_subrounds_mixed_calls(r, mode, policy):
    say(f"sub-rounds {r}: {mode} {policy}")
    nb = 16
    tw = Twin(nb * 128, 8, mode, policy, seed=r)
    tw.gpu.set_route_subrounds(r)
    tw.ora.set_subrounds(r)
    assert tw.gpu.route_subrounds == r
    rng = np.random.default_rng(r * 7 + len(mode) + len(policy))
    universe = np.concatenate([np_keys(70 + r, nb * 128 * 3), np.array([0, M64], dtype=np.uint64)])

    def scores(n):
        if policy == "custom":
            return rng.integers(0, 40, n).astype(np.uint64)
        if policy == "lfu":
            return rng.choice(np.array([1, 1, 2, 9], dtype=np.uint64), n)
        return None

    for step in range(20):
        n = int(rng.integers(0, nb * 128 * 2))
        k = rng.choice(universe, n)
        x = step % 5
        if x in (0, 1):
            tw.upsert(k, scores(n), evict=x == 1)
        elif x == 2:
            tw.find_or_insert(k, scores(n))
        elif x == 3:
            tw.find(k)
        else:
            tw.erase(k[: n // 3])
        tw.check_table()


def test_subrounds_place_a_large_batch():
    """One call of 0.95 x capacity fresh keys into an empty dual table: with one round the
    snapshot sends every key to b1 and some are refused; 64 sub-rounds place all of them."""
    placed = {}
    for r in (1, 64):
        say(f"large fresh batch, sub-rounds {r}")
        tw = Twin(64 * 128, 8, "dual", "custom", seed=1)
        tw.gpu.set_route_subrounds(r)
        tw.ora.set_subrounds(r)
        n = int(0.95 * 64 * 128)
        st = tw.upsert(np_keys(80, n), np.full(n, 1, dtype=np.uint64))
        tw.check_table()
        placed[r] = float((st == cskv.ST_INSERTED).mean())
    assert placed[1] < 0.99 and placed[64] == 1.0


@pytest.mark.parametrize("overlap", [0, 1, 2])
def test_subround_programs_match_calls(overlap):
    say(f"programs with sub-rounds, overlap {overlap}")
    cap, dim, r = 1 << 15, 8, 4
    tables = [prefilled(cap, dim, 24000) for _ in range(3)]
    for t in tables:
        t.set_route_subrounds(r)
    base, t_prog, t_graph = tables
    resident = gen_keys(1, 24000, device="cuda")
    sched = batch_schedule(9, 40, 16, 4096)
    ops = program_inputs(sched, dim, resident, fresh_stream=42, miss_stream=43, seed=3, device="cuda")
    run_calls(base, ops)
    torch.cuda.synchronize()
    ops_p = fresh_outputs(ops)
    prog = build_program(t_prog, ops_p, overlap=overlap)
    prog.launch()
    torch.cuda.synchronize()
    same_outputs(ops, ops_p)
    same_tables(base, t_prog)
    ops_g = fresh_outputs(ops)
    prog_g = build_program(t_graph, ops_g, overlap=overlap)
    s = torch.cuda.Stream()
    prog_g.capture(s)
    prog_g.replay(s)
    s.synchronize()
    same_outputs(ops, ops_g)
    same_tables(base, t_graph)
    # a program built for r sub-rounds refuses to run once the table's setting changed
    t_prog.set_route_subrounds(1)
    with pytest.raises(cskv.CskvError):
        prog.launch()
    torch.cuda.synchronize()


def test_subround_bounds():
    t = cskv.Table(128 * 4, 8, "dual", "custom")
    for bad in (0, 65):
        with pytest.raises(cskv.CskvError):
            t.set_route_subrounds(bad)
    t.set_route_subrounds(64)
    assert t.route_subrounds == 64
