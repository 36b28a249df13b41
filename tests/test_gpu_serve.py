"""Serving loop: every request's result is the same alone (issued by itself, in admission order)
and in the mix (merged reader launches, overlapping groups, reader groups on streams of their own
running concurrently, budget-deferred admission), and equals the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2603_17168_amd import cskv, serve
from paper_2603_17168_amd.workload import (Zipf, as_u64, from_u64, keys as gen_keys, lognormal_sizes,
                                            poisson_arrivals, uniform01, value_rows)
from tests.parity import bits

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_trace(table, nreq, seed, qps, zipf_n=1 << 20):
    sizes = lognormal_sizes(seed, nreq, 256.0, 1.0, 16, 4096)
    ops = np.where(uniform01(seed + 1, nreq).numpy() < 0.9, serve.REQ_FIND, serve.REQ_INSERT_AND_EVICT)
    z = Zipf(1.1, zipf_n).sample(seed + 2, int(sizes.sum()))
    keys = from_u64(z, "cuda")
    ins = ops == serve.REQ_INSERT_AND_EVICT
    off = np.concatenate([[0], np.cumsum(sizes)])
    ins_keys = torch.cat([keys[off[i]:off[i + 1]] for i in range(nreq) if ins[i]] or
                         [torch.zeros(0, dtype=torch.int64, device="cuda")])
    vals = value_rows(5, ins_keys, table.dim)  # value id = key
    arr = poisson_arrivals(seed + 3, nreq, qps)
    return ops, sizes, keys, vals, arr


def prefill(table, n, batch=1 << 13):
    ks = []
    for s in range(0, n, batch):
        k = torch.arange(1 + s, 1 + s + min(batch, n - s), dtype=torch.int64, device="cuda")
        table.insert_or_assign(k, value_rows(5, k, table.dim), want_status=False)
        ks.append(k)
    torch.cuda.synchronize()
    return torch.cat(ks)


def clone(src):
    dst = cskv.Table(src.capacity, src.dim, mode=src.mode, policy=src.policy)
    dst.storage.copy_(src.storage)
    torch.cuda.synchronize()
    return dst


@pytest.mark.parametrize("streams", [0, 2])
@pytest.mark.parametrize("mode", ["realtime", "burst", "tight_budget"])
def test_serving_alone_equals_mix_and_oracle(mode, streams):
    cap, dim = 1 << 15, 16
    base = cskv.Table(cap, dim, "dual", "lru")
    pre = prefill(base, 30000)
    alone = clone(base)
    ora = oracle.Oracle(cap // 128, 128, oracle.DUAL, oracle.LRU)
    pk = as_u64(pre.cpu())
    for s in range(0, pk.size, 1 << 13):
        ora.upsert(pk[s:s + (1 << 13)], pk[s:s + (1 << 13)])
    nreq = 160
    ops, sizes, keys, vals, arr = make_trace(base, nreq, seed=11, qps=20000.0)
    tr = serve.Trace(base, ops, sizes, keys, vals, arr, with_results=True)
    budget = 1 << 20 if mode == "tight_budget" else 256 << 20
    say(f"serving {nreq} requests, mode {mode}, reader streams {streams}")
    stats, times = serve.serve(base, tr, budget_bytes=budget, max_inflight_groups=4 if streams else 2, max_merge=16,
                               realtime=(mode == "realtime"), reader_streams=streams)
    say(stats)
    assert stats["completed"] == nreq
    assert np.array_equal(times["seq"], np.arange(nreq))  # admission order = arrival order
    assert (times["complete_s"] >= times["launch_s"]).all() and (times["launch_s"] >= times["admit_s"]).all()
    if mode == "burst":
        assert stats["reader_launches"] < (ops == serve.REQ_FIND).sum()  # finds were merged
    if mode == "tight_budget":
        assert stats["deferred_for_memory"] > 0 and stats["peak_inflight_bytes"] <= budget
    # each request alone, in admission order, on the starting table; and the oracle
    koff = tr.key_off
    for i in np.argsort(times["seq"]):
        k = keys[koff[i]:koff[i + 1]]
        kk = as_u64(k.cpu())
        if ops[i] == serve.REQ_FIND:
            v, f, _ = alone.find(k, want_scores=False)
            o = tr.find_off[i]
            assert torch.equal(f, tr.find_flag[o:o + sizes[i]])
            hit = f.bool()
            assert torch.equal(bits(v[hit]), bits(tr.find_out[o:o + sizes[i]][hit]))
            of, ov, _ = ora.find(kk)
            assert np.array_equal(f.cpu().numpy(), of)
            h = np.nonzero(of)[0]
            if h.size:
                exp = value_rows(5, torch.from_numpy(ov[h].view(np.int64)), dim)
                assert torch.equal(bits(v.cpu()[torch.from_numpy(h)]), bits(exp))
        else:
            o = tr.val_off[i]
            st, ek, ev, es, cnt = alone.insert_and_evict(k, vals[o:o + sizes[i]])
            assert torch.equal(st, tr.ins_status[o:o + sizes[i]])
            m = int(cnt.item())
            assert m == int(tr.ev_count[i].item())
            a = torch.argsort(ek[:m])
            b = torch.argsort(tr.ev_keys[o:o + m])
            assert torch.equal(ek[:m][a], tr.ev_keys[o:o + m][b])
            assert torch.equal(es[:m][a], tr.ev_scores[o:o + m][b])
            assert torch.equal(bits(ev[:m][a]), bits(tr.ev_vals[o:o + m][b]))
            ost, oek, oev, oes = ora.upsert(kk, kk)
            assert np.array_equal(st.cpu().numpy(), ost)
            assert np.array_equal(np.sort(as_u64(ek[:m].cpu())), np.sort(oek))
    assert alone.size() == base.size() == ora.size()
