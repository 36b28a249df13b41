"""Seeded synthetic input generators shared by the GPU path's tests/bench and the oracle's tests.

This module holds no arithmetic of the hash table itself (no bucket hash, no routing, no
eviction): only the counter-based random streams that produce the workloads' keys, scores,
value rows and request mixes.  Every generator is a pure function of (seed, counter), so the
same call yields the same numbers on the CPU and on a GPU tensor.

Streams used (all 64-bit, wrapping arithmetic):
  * ``mix64`` - the output function of Vigna's SplitMix64 generator (public domain), a bijection
    on 64-bit words.  Keys are ``mix64(stream << 40 | i)``, so keys drawn from distinct counters
    are distinct.  The two reserved key words (0 and 2**64-1) are replaced by ``mix64(~counter)``.
  * value rows: element j of the row with value-id ``v`` is ``u24 * 2**-23 - 1`` where ``u24`` is
    the top 24 bits of ``mix64(mix64(seed_word ^ v) + j)``; every element is an exactly
    representable float32 in [-1, 1).
  * Zipf ranks by rejection-inversion (Hormann & Derflinger, 1996).

torch int64 tensors stand in for unsigned 64-bit words: multiplication and addition wrap, and
logical right shifts are done with a mask.
"""
from __future__ import annotations

import math

import numpy as np
import torch

_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_GOLD = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


def _s64(x: int) -> int:
    """Two's-complement int64 view of an unsigned 64-bit python int."""
    x &= MASK64
    return x - (1 << 64) if x >= (1 << 63) else x


def _lsr(x: torch.Tensor, k: int) -> torch.Tensor:
    return (x >> k) & ((1 << (64 - k)) - 1)


def mix64(x: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output function on an int64 tensor (bit pattern of uint64)."""
    z = x
    z = (z ^ _lsr(z, 30)) * _s64(_M1)
    z = (z ^ _lsr(z, 27)) * _s64(_M2)
    return z ^ _lsr(z, 31)


def mix64_int(x: int) -> int:
    """Scalar reference of :func:`mix64` on python ints."""
    z = x & MASK64
    z = ((z ^ (z >> 30)) * _M1) & MASK64
    z = ((z ^ (z >> 27)) * _M2) & MASK64
    return z ^ (z >> 31)


def keys(stream: int, n: int, start: int = 0, device="cpu") -> torch.Tensor:
    """n distinct, nonzero, non-all-ones u64 keys (as int64) from key stream ``stream``.

    Distinct streams (< 2**24) and distinct counters (< 2**40) give distinct keys, because
    mix64 is a bijection.
    """
    assert 0 <= stream < (1 << 24) and 0 <= start and start + n <= (1 << 40)
    ctr = torch.arange(start, start + n, dtype=torch.int64, device=device) | _s64(stream << 40)
    k = mix64(ctr)
    bad = (k == 0) | (k == -1)
    if bool(bad.any()):
        k = torch.where(bad, mix64(~ctr), k)
    return k


def keys_at(stream: int, counters: torch.Tensor) -> torch.Tensor:
    """The keys of stream `stream` at arbitrary counters (< 2**40): keys(stream, n, start) is
    keys_at(stream, arange(start, start + n))."""
    ctr = counters.to(torch.int64) | _s64(stream << 40)
    k = mix64(ctr)
    bad = (k == 0) | (k == -1)
    if bool(bad.any()):
        k = torch.where(bad, mix64(~ctr), k)
    return k


def value_rows(seed: int, vids: torch.Tensor, dim: int) -> torch.Tensor:
    """float32 rows [len(vids), dim]; row r is a pure function of (seed, vids[r])."""
    vids = vids.to(torch.int64)
    base = mix64(vids ^ _s64(mix64_int(seed * _GOLD + 1)))
    j = torch.arange(dim, dtype=torch.int64, device=vids.device)
    z = mix64(base[:, None] + j[None, :])
    u24 = _lsr(z, 40).to(torch.float64)
    return (u24 * (2.0 ** -23) - 1.0).to(torch.float32)


def uniform_u64(stream: int, n: int, start: int = 0, device="cpu") -> torch.Tensor:
    """n uniform 64-bit words (int64 view) from a counter stream; may repeat across streams."""
    ctr = torch.arange(start, start + n, dtype=torch.int64, device=device)
    return mix64(mix64(ctr ^ _s64(mix64_int(stream * _GOLD + 7))))


def uniform01(stream: int, n: int, start: int = 0, device="cpu") -> torch.Tensor:
    """n float64 uniforms in [0, 1) with 53 random bits each."""
    w = uniform_u64(stream, n, start, device)
    return _lsr(w, 11).to(torch.float64) * (2.0 ** -53)


def randint(stream: int, n: int, hi: int, start: int = 0, device="cpu") -> torch.Tensor:
    """n integers uniform in [0, hi) (hi < 2**53), int64."""
    return torch.floor(uniform01(stream, n, start, device) * hi).to(torch.int64)


def permutation(stream: int, n: int) -> torch.Tensor:
    """A seeded permutation of range(n) (argsort of uniform words)."""
    return torch.argsort(uniform_u64(stream, n))


class Zipf:
    """Zipf(alpha) ranks in [1, N] by rejection-inversion (Hormann & Derflinger 1996).

    P(rank = k) is proportional to k**-alpha.  Vectorised over a counter stream of uniforms;
    rejected draws are redrawn from a second counter range of the same stream.
    """

    def __init__(self, alpha: float, n_max: int):
        assert alpha > 0 and alpha != 1.0 and n_max >= 1
        self.a = float(alpha)
        self.N = int(n_max)
        self.h_x1 = self._H(1.5) - 1.0
        self.h_n = self._H(self.N + 0.5)
        self.s = 2.0 - self._Hinv(self._H(2.5) - 2.0 ** -self.a)

    def _H(self, x):
        # integral of x**-a: (x**(1-a) - 1) / (1-a), written with expm1/log1p for accuracy
        return np.expm1((1.0 - self.a) * np.log(x)) / (1.0 - self.a)

    def _Hinv(self, y):
        t = np.maximum(y * (1.0 - self.a), -1.0 + 1e-300)
        return np.exp(np.log1p(t) / (1.0 - self.a))

    def sample_device(self, stream: int, n: int, device) -> torch.Tensor:
        """The same algorithm in float64 torch ops on `device` (int64 ranks); seeded, but not
        guaranteed to equal :meth:`sample` draw for draw (libm rounding may differ)."""
        a = self.a
        H = lambda x: torch.expm1((1.0 - a) * torch.log(x)) / (1.0 - a)
        Hinv = lambda y: torch.exp(torch.log1p(torch.clamp(y * (1.0 - a), min=-1.0 + 1e-300)) / (1.0 - a))
        out = torch.empty(n, dtype=torch.int64, device=device)
        todo = torch.arange(n, device=device)
        ctr = 0
        while todo.numel():
            u = uniform01(stream, todo.numel(), start=ctr, device=device)
            ctr += todo.numel()
            u = self.h_n + u * (self.h_x1 - self.h_n)
            x = Hinv(u)
            k = torch.clamp(torch.floor(x + 0.5), 1, self.N)
            ok = (k - x <= self.s) | (u >= H(k + 0.5) - torch.exp(-a * torch.log(k)))
            out[todo[ok]] = k[ok].to(torch.int64)
            todo = todo[~ok]
        return out

    def sample(self, stream: int, n: int) -> np.ndarray:
        out = np.empty(n, dtype=np.uint64)
        todo = np.arange(n)
        ctr = 0
        while todo.size:
            u = uniform01(stream, todo.size, start=ctr).numpy()
            ctr += todo.size
            u = self.h_n + u * (self.h_x1 - self.h_n)
            x = self._Hinv(u)
            k = np.clip(np.floor(x + 0.5), 1, self.N)
            ok = (k - x <= self.s) | (u >= self._H(k + 0.5) - np.exp(-self.a * np.log(k)))
            out[todo[ok]] = k[ok].astype(np.uint64)
            todo = todo[~ok]
        return out


def as_u64(t: torch.Tensor) -> np.ndarray:
    """int64 tensor -> numpy uint64 array (same bits)."""
    return t.detach().cpu().numpy().view(np.uint64)


def from_u64(a, device="cpu") -> torch.Tensor:
    """numpy uint64 array -> int64 tensor (same bits)."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint64)).view(np.int64)).to(device)


def lognormal_sizes(stream: int, n: int, median: float, sigma: float, lo: int, hi: int) -> np.ndarray:
    """Request sizes: lognormal(median, sigma) clipped to [lo, hi] (Box-Muller on counter uniforms)."""
    u1 = uniform01(stream, n).numpy()
    u2 = uniform01(stream, n, start=n).numpy()
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)
    return np.clip(np.round(median * np.exp(sigma * z)), lo, hi).astype(np.int64)


def poisson_arrivals(stream: int, n: int, rate_per_s: float) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: cumulative exponential gaps."""
    u = uniform01(stream, n).numpy()
    return np.cumsum(-np.log1p(-u) / rate_per_s)


def batch_schedule(stream: int, nbatches: int, lo: int, hi: int, mix=(0.70, 0.25, 0.05)):
    """Uneven batch program: sizes log-uniform in [lo, hi], ops drawn find / insert_or_assign /
    erase with probabilities `mix`.  Returns a list of (op, size) with op in {"find", "upsert",
    "erase"}."""
    u = uniform01(stream, 2 * nbatches).numpy()
    sizes = np.floor(np.exp(np.log(lo) + u[:nbatches] * (np.log(hi) - np.log(lo)))).astype(np.int64)
    sizes = np.clip(sizes, lo, hi)
    ops = []
    c1, c2 = mix[0], mix[0] + mix[1]
    for i in range(nbatches):
        r = u[nbatches + i]
        ops.append(("find" if r < c1 else "upsert" if r < c2 else "erase", int(sizes[i])))
    return ops


def program_inputs(schedule, dim: int, resident: torch.Tensor, fresh_stream: int, miss_stream: int, seed: int,
                   device="cpu"):
    """Device inputs and output buffers for a batch schedule (see :func:`batch_schedule`).

    find: half the keys drawn with replacement from `resident`, half never-inserted keys from
    `miss_stream`, shuffled; upsert: fresh keys from `fresh_stream` with rows from `value_rows`;
    erase: keys drawn from `resident`.  Returns a list of dicts with the op, its inputs and
    freshly allocated outputs."""
    out = []
    fresh_ctr = 0
    miss_ctr = 0
    nres = resident.numel()
    for j, (op, n) in enumerate(schedule):
        d = {"op": op, "n": n}
        if op == "find":
            h = n // 2
            idx = randint(10_000 + j, n - h, nres, device=device)
            miss = keys(miss_stream, h, miss_ctr, device=device)
            miss_ctr += h
            q = torch.cat([resident.to(device)[idx], miss])
            perm = torch.argsort(uniform_u64(20_000 + j, n, device=device))
            d["keys"] = q[perm].contiguous()
            d["out"] = torch.zeros((n, dim), dtype=torch.float32, device=device)
            d["flag"] = torch.empty(n, dtype=torch.uint8, device=device)
        elif op == "upsert":
            k = keys(fresh_stream, n, fresh_ctr, device=device)
            fresh_ctr += n
            d["keys"] = k
            d["values"] = value_rows(seed, k, dim)
            d["flag"] = torch.empty(n, dtype=torch.uint8, device=device)
        else:
            idx = randint(30_000 + j, n, nres, device=device)
            d["keys"] = resident.to(device)[idx].contiguous()
            d["flag"] = torch.empty(n, dtype=torch.uint8, device=device)
        out.append(d)
    return out
