"""GPU-vs-oracle parity harness: drives the HIP table (through the C-ABI binding) and the
sequential C oracle with identical seeded inputs and compares every output bit for bit.

Value rows are generated from value-ids by the shared seeded generator; the oracle stores
value-ids, the GPU stores the rows, and rows are compared as raw 32-bit patterns.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2603_17168_amd import cskv
from paper_2603_17168_amd.workload import as_u64, from_u64, value_rows

MODE = {"single": oracle.SINGLE, "dual": oracle.DUAL}
POLICY = {"custom": oracle.CUSTOM, "lru": oracle.LRU, "lfu": oracle.LFU}
NAN_BITS = 0x7FC0DEAD


def bits(t: torch.Tensor) -> torch.Tensor:
    return t.contiguous().view(torch.int32)


class Twin:
    def __init__(self, capacity: int, dim: int, mode: str = "dual", policy: str = "custom", seed: int = 1,
                 device="cuda", hbm_value_rows=None):
        self.gpu = cskv.Table(capacity, dim, mode=mode, policy=policy, device=device, hbm_value_rows=hbm_value_rows)
        self.ora = oracle.Oracle(capacity // 128, 128, MODE[mode], POLICY[policy])
        self.dim = dim
        self.seed = seed
        self.device = self.gpu.device
        self.next_vid = 1
        self.policy = policy

    def rows(self, vids: np.ndarray) -> torch.Tensor:
        return value_rows(self.seed, torch.from_numpy(np.asarray(vids, dtype=np.uint64).view(np.int64)), self.dim)

    def _vids(self, n: int) -> np.ndarray:
        v = np.arange(self.next_vid, self.next_vid + n, dtype=np.uint64)
        self.next_vid += n
        return v

    # ------------------------------------------------------------------ operations
    def upsert(self, keys: np.ndarray, scores: np.ndarray | None = None, evict: bool = False, check=True):
        keys = np.asarray(keys, dtype=np.uint64)
        n = keys.size
        vids = self._vids(n)
        kd = from_u64(keys, self.device)
        vd = self.rows(vids).to(self.device)
        sd = None if scores is None else from_u64(np.asarray(scores, dtype=np.uint64), self.device)
        if evict:
            st, ek, ev, es, cnt = self.gpu.insert_and_evict(kd, vd, sd)
        else:
            st = self.gpu.insert_or_assign(kd, vd, sd)
        ost, oek, oev, oes = self.ora.upsert(keys, vids, scores)
        if not check:
            return ost
        torch.cuda.synchronize()
        gst = st.cpu().numpy()
        if not np.array_equal(gst, ost):
            bad = np.nonzero(gst != ost)[0]
            raise AssertionError(f"status mismatch at {bad[:10]}: gpu {gst[bad[:10]]} oracle {ost[bad[:10]]}")
        if evict:
            m = int(cnt.item())
            assert m == oek.size, f"evicted count gpu {m} oracle {oek.size}"
            gk = as_u64(ek[:m])
            order = np.argsort(gk, kind="stable")
            oorder = np.argsort(oek, kind="stable")
            assert np.array_equal(gk[order], oek[oorder]), "evicted keys differ"
            assert np.array_equal(as_u64(es[:m])[order], oes[oorder]), "evicted scores differ"
            if m:
                got = bits(ev[:m].cpu()[torch.from_numpy(order)])
                exp = bits(self.rows(oev[oorder]))
                assert torch.equal(got, exp), "evicted rows differ"
        assert self.gpu.clock == self.ora.clock
        return ost

    def find(self, keys: np.ndarray):
        keys = np.asarray(keys, dtype=np.uint64)
        n = keys.size
        kd = from_u64(keys, self.device)
        out = torch.full((n, self.dim), 0, dtype=torch.int32, device=self.device)
        out.fill_(NAN_BITS)
        out = out.view(torch.float32)
        vals, found, sc = self.gpu.find(kd, values_out=out)
        of, ov, osc = self.ora.find(keys)
        torch.cuda.synchronize()
        gf = found.cpu().numpy()
        assert np.array_equal(gf, of), f"found mask differs at {np.nonzero(gf != of)[0][:10]}"
        hit = np.nonzero(of)[0]
        miss = np.nonzero(of == 0)[0]
        gv = bits(vals.cpu())
        if hit.size:
            assert torch.equal(gv[torch.from_numpy(hit)], bits(self.rows(ov[hit]))), "found rows differ"
            assert np.array_equal(as_u64(sc.cpu())[hit], osc[hit]), "found scores differ"
        if miss.size:
            assert bool((gv[torch.from_numpy(miss)] == NAN_BITS).all()), "rows of missing keys were written"
        return of

    def erase(self, keys: np.ndarray):
        keys = np.asarray(keys, dtype=np.uint64)
        er = self.gpu.erase(from_u64(keys, self.device))
        oer = self.ora.erase(keys)
        torch.cuda.synchronize()
        assert np.array_equal(er.cpu().numpy(), oer), "erased flags differ"
        return oer

    def _scores_arg(self, scores):
        return None if scores is None else from_u64(np.asarray(scores, dtype=np.uint64), self.device)

    def contains(self, keys: np.ndarray):
        keys = np.asarray(keys, dtype=np.uint64)
        f = self.gpu.contains(from_u64(keys, self.device))
        of = self.ora.contains(keys)
        torch.cuda.synchronize()
        assert np.array_equal(f.cpu().numpy(), of), "contains flags differ"
        return of

    def find_ptr(self, keys: np.ndarray):
        """Pointers must address the resident row: one base for all, each slot in the oracle's
        bucket for the key, rows equal (via the slot -> row map of the exported table)."""
        keys = np.asarray(keys, dtype=np.uint64)
        sc = torch.empty(keys.size, dtype=torch.int64, device=self.device)
        ptr, f, sc = self.gpu.find_ptr(from_u64(keys, self.device), scores_out=sc)
        of, ob = self.ora.locate(keys)
        _, _, osc = self.ora.find(keys)
        torch.cuda.synchronize()
        assert np.array_equal(f.cpu().numpy(), of), "find_ptr flags differ"
        gp = as_u64(ptr)
        hit = np.nonzero(of)[0]
        assert np.all(gp[of == 0] == 0), "absent keys got a pointer"
        if hit.size == 0:
            return of
        gk, gv, gs, gsl = self.gpu.export()
        slot_of = dict(zip(as_u64(gk).tolist(), as_u64(gsl).tolist()))
        rb = self.dim * 4
        hbm = self.gpu.hbm_value_rows
        hbm_base = self.gpu.row_address(0) if hbm > 0 else None
        host_base = self.gpu.row_address(hbm) if hbm < self.gpu.capacity else None
        store = self.gpu.storage.cpu()
        host = None if self.gpu.host_values is None else self.gpu.host_values.view(torch.int32)
        _, ov, _ = self.ora.find(keys)
        for i in hit:
            sl = slot_of[int(keys[i])]
            # position-based addressing: one linear map per storage region
            want = hbm_base + sl * rb if sl < hbm else host_base + (sl - hbm) * rb
            assert int(gp[i]) == want, "pointer does not address the key's slot"
            assert sl // 128 == int(ob[i]), "pointer outside the key's bucket"
            if sl < hbm:  # the row at the pointer is the key's row
                off = int(gp[i]) - self.gpu.storage.data_ptr()
                got = store[off:off + rb].view(torch.int32)
            else:
                got = host[(sl - hbm) * self.dim:(sl - hbm + 1) * self.dim]
            assert torch.equal(got, bits(self.rows(ov[i:i + 1]))[0]), "the row at the pointer differs"
        assert np.array_equal(as_u64(sc.cpu())[hit], osc[hit]), "find_ptr scores differ"
        return of

    def assign(self, keys: np.ndarray, scores=None, with_values: bool = True):
        keys = np.asarray(keys, dtype=np.uint64)
        kd = from_u64(keys, self.device)
        if with_values:
            vids = self._vids(keys.size)
            f = self.gpu.assign(kd, self.rows(vids).to(self.device), self._scores_arg(scores))
            of = self.ora.assign(keys, vids, scores)
        else:
            f = self.gpu.assign_scores(kd, self._scores_arg(scores))
            of = self.ora.assign(keys, None, scores)
        torch.cuda.synchronize()
        assert np.array_equal(f.cpu().numpy(), of), "assign flags differ"
        assert self.gpu.clock == self.ora.clock
        return of

    def find_or_insert(self, keys: np.ndarray, scores=None):
        keys = np.asarray(keys, dtype=np.uint64)
        n = keys.size
        vids = self._vids(n)
        out = torch.full((n, self.dim), 0, dtype=torch.int32, device=self.device)
        out.fill_(NAN_BITS)
        out = out.view(torch.float32)
        vals, st = self.gpu.find_or_insert(from_u64(keys, self.device), self.rows(vids).to(self.device),
                                           self._scores_arg(scores), values_out=out)
        ost, ovid = self.ora.find_or_insert(keys, vids, scores)
        torch.cuda.synchronize()
        gst = st.cpu().numpy()
        if not np.array_equal(gst, ost):
            bad = np.nonzero(gst != ost)[0]
            raise AssertionError(f"find_or_insert status mismatch at {bad[:10]}: gpu {gst[bad[:10]]} oracle {ost[bad[:10]]}")
        valid = np.nonzero(ost != oracle.INVALID_KEY)[0]
        bad_rows = np.nonzero(ost == oracle.INVALID_KEY)[0]
        gv = bits(vals.cpu())
        if valid.size:
            assert torch.equal(gv[torch.from_numpy(valid)], bits(self.rows(ovid[valid]))), "find_or_insert rows differ"
        if bad_rows.size:
            assert bool((gv[torch.from_numpy(bad_rows)] == NAN_BITS).all()), "rows of reserved keys were written"
        assert self.gpu.clock == self.ora.clock
        return ost

    def export_if(self, min_score: int):
        gk, gv, gs, gsl = self.gpu.export(min_score=min_score)
        ok, ov, os_, ob = self.ora.export_if(min_score)
        torch.cuda.synchronize()
        gk = as_u64(gk)
        assert gk.size == ok.size, f"export_if count gpu {gk.size} oracle {ok.size}"
        go, oo = np.argsort(gk, kind="stable"), np.argsort(ok, kind="stable")
        assert np.array_equal(gk[go], ok[oo]) and np.array_equal(as_u64(gs)[go], os_[oo])
        if gk.size:
            assert torch.equal(bits(gv.cpu()[torch.from_numpy(go)]), bits(self.rows(ov[oo]))), "export_if rows differ"

    # ------------------------------------------------------------------ whole-table check
    def check_table(self, with_values: bool = True):
        gk, gv, gs, gsl = self.gpu.export(with_values=with_values)
        torch.cuda.synchronize()
        ok, ov, os_, ob = self.ora.export()
        gk = as_u64(gk)
        assert gk.size == ok.size, f"table size gpu {gk.size} oracle {ok.size}"
        assert self.gpu.size() == ok.size
        go = np.argsort(gk, kind="stable")
        oo = np.argsort(ok, kind="stable")
        assert np.array_equal(gk[go], ok[oo]), "table keys differ"
        assert np.array_equal(as_u64(gs)[go], os_[oo]), "table scores differ"
        gslots = as_u64(gsl)
        assert np.unique(gslots).size == gslots.size, "two entries share a slot"
        assert np.array_equal((gslots // 128)[go], ob[oo]), "an entry sits in a different bucket"
        if with_values and gk.size:
            got = bits(gv.cpu()[torch.from_numpy(go)])
            exp = bits(self.rows(ov[oo]))
            assert torch.equal(got, exp), "table rows differ"
