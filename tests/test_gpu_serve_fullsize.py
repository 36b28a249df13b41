"""The serving loop at the bench's C5 size (2^28 slots, dim 128, LRU, ~142 GB, prefilled with
ranks 1..2^28; lognormal(4096, 1.0) request sizes, 90 % find / 10 % insert_and_evict, Zipf(1.1)
keys over 2^34; continuous batching), checked by properties that hold whatever the serialization
order: every row written or read equals its generator row (prefill and inserts use the same
one), statuses and evicted counts agree, evicted rows are their keys' rows, and the keys of the
last insert in serialization order are resident at the end.  The order itself and exact results
are checked against the oracle at small size (test_gpu_serve.py)."""
import sys

import numpy as np
import pytest
import torch

from paper_2603_17168_amd import cskv, serve
from paper_2603_17168_amd.workload import Zipf, lognormal_sizes, uniform01, value_rows

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bits(t):
    return t.contiguous().view(torch.int32)


def test_c5_serving_full_size_properties():
    dev = torch.device("cuda", 0)
    cap, dim, nreq = 1 << 28, 128, 2000
    say("C5 full size: prefill 2^28 slots, dim 128")
    t = cskv.Table(cap, dim, mode="dual", policy="lru", device=dev)
    b = 1 << 20
    for s0 in range(0, cap, b):
        k = torch.arange(1 + s0, 1 + s0 + b, dtype=torch.int64, device=dev)
        t.insert_or_assign(k, value_rows(13, k, dim), want_status=False)
    size0 = t.size()
    assert size0 > 0.99 * cap
    sizes = lognormal_sizes(31, nreq, 4096.0, 1.0, 256, 65536)
    ops = np.where(uniform01(32, nreq).numpy() < 0.9, serve.REQ_FIND, serve.REQ_INSERT_AND_EVICT)
    keys = Zipf(1.1, 1 << 34).sample_device(33, int(sizes.sum()), dev)
    ins = ops == serve.REQ_INSERT_AND_EVICT
    off = np.concatenate([[0], np.cumsum(sizes)])
    ins_keys = torch.cat([keys[off[i]:off[i + 1]] for i in range(nreq) if ins[i]])
    vals = value_rows(13, ins_keys, dim)  # the prefill's generator: every resident row is f(key)
    tr = serve.Trace(t, ops, sizes, keys, vals, np.zeros(nreq), with_results=True)
    say(f"serve {nreq} requests, {int(sizes.sum())} keys")
    st, times = serve.serve(t, tr, 4 << 30, max_inflight_groups=2, max_merge=64, realtime=False)
    assert st["groups"] > 0 and st["groups"] < nreq  # finds were merged
    say("check finds")
    fk = torch.cat([keys[off[i]:off[i + 1]] for i in range(nreq) if not ins[i]])
    ff = tr.find_flag[: fk.numel()].bool()
    assert 0.5 < float(ff.float().mean()) < 1.0
    for c in range(0, fk.numel(), 1 << 20):
        sel = ff[c:c + (1 << 20)]
        got = tr.find_out[c:c + (1 << 20)][sel]
        assert torch.equal(bits(got), bits(value_rows(13, fk[c:c + (1 << 20)][sel], dim))), "a found row differs"
    say("check inserts")
    ist = tr.ins_status[: ins_keys.numel()]
    assert bool(((ist >= cskv.ST_UPDATED) & (ist <= cskv.ST_REJECTED)).all())
    io = np.concatenate([[0], np.cumsum(sizes[ins])])
    ev_total = 0
    for j, i in enumerate(np.nonzero(ins)[0]):
        s_ = ist[io[j]:io[j + 1]]
        m = int(tr.ev_count[i].item())
        # one eviction per distinct key admitted into a full bucket (repeats share the status)
        kk = ins_keys[io[j]:io[j + 1]]
        assert m == torch.unique(kk[s_ == cskv.ST_INSERTED_EVICT]).numel(), f"request {i}: evicted count"
        ek = tr.ev_keys[io[j]:io[j] + m]
        assert torch.unique(ek).numel() == m
        assert torch.equal(bits(tr.ev_vals[io[j]:io[j] + m]), bits(value_rows(13, ek, dim))), "an evicted row differs"
        ev_total += m
    assert ev_total > 0
    # the last insert in serialization order: its admitted keys are resident at the end
    seq = times["seq"]
    last = max(np.nonzero(ins)[0], key=lambda i: seq[i])
    j = int(np.nonzero(np.nonzero(ins)[0] == last)[0][0])
    lk = ins_keys[io[j]:io[j + 1]]
    ls = ist[io[j]:io[j + 1]]
    adm = (ls == cskv.ST_UPDATED) | (ls == cskv.ST_INSERTED) | (ls == cskv.ST_INSERTED_EVICT)
    v, f, _ = t.find(lk[adm])
    assert bool((f == 1).all()) and torch.equal(bits(v), bits(value_rows(13, lk[adm], dim)))
    del t, tr, keys, vals
    torch.cuda.empty_cache()
