"""Tile plans against a host replay of the planning rule ("Parallelization":
consecutive whole intervals per tile, never split; an interval beyond a
tile's capacity gets a tile of its own). The per-interval block and value
counts come from the oracle's conversion, the rule is replayed here, and
the library's tile and long-tile counts must match exactly:
  * modes 0 and 1: at most cap / (r c) blocks per tile, where cap is
    (64 chunks - 1) * 16 / value size mask bits (mode 0) or tile_bits
    (mode 1); at most 127 intervals for r = 1, else 128 / r (mode 0) or
    256 / r (mode 1);
  * modes 3 and 4 (lanes on value-sized tiles): at most (64 chunks - 1) *
    16 / value size values and at most min(4032 / (r c), 128 chunks / r -
    64 / (r c) + 1) blocks per tile, the intervals capped as in mode 0.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1801_01134_amd as spc
from paper_1801_01134_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


MATS = {
    "stencil16": lambda: synth.stencil27(16),
    "powerlaw": lambda: synth.powerlaw(3001, 3001, seed=2),
    "uniform": lambda: synth.uniform_random(5000, 4000, 12.0, seed=7),
    "band": lambda: synth.band_plus_uniform(4096, seed=0),
    "diagonal": lambda: synth.from_keys_sorted(6007, 6007, np.arange(6007), np.arange(6007), 11),
    "dense_rows": lambda: synth.from_keys_sorted(
        300, 9000, np.repeat(np.array([3, 4, 250]), 9000), np.tile(np.arange(9000), 3), 13),
}
_cache = {}


def mat(name):
    if name not in _cache:
        _cache[name] = MATS[name]()
    return _cache[name]


def interval_counts(A, r, c):
    ref = oracle.csr_to_beta(A, r, c)
    brp = np.asarray(ref.block_rowptr, dtype=np.int64)
    blocks = np.diff(brp)
    pc = np.array([bin(int(m)).count("1") for m in ref.masks], dtype=np.int64)
    cum = np.concatenate([[0], np.cumsum(pc)])
    values = cum[brp[1:]] - cum[brp[:-1]]
    return blocks, values


def replay(blocks, values, nb_cap, v_cap, max_int):
    n_tiles = n_long = 0
    i, n = 0, len(blocks)
    while i < n:
        if blocks[i] > nb_cap or values[i] > v_cap:
            n_tiles += 1
            n_long += 1
            i += 1
            continue
        start, b, v = i, 0, 0
        while i < n and i - start < max_int:
            if blocks[i] > nb_cap or values[i] > v_cap or b + blocks[i] > nb_cap or v + values[i] > v_cap:
                break
            b += blocks[i]
            v += values[i]
            i += 1
        n_tiles += 1
    return n_tiles, n_long


@pytest.mark.parametrize("rc", spc.SHAPES, ids=lambda s: f"b{s[0]}x{s[1]}")
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_plan_counts_match_the_rule(rc, dtype):
    r, c = rc
    say(f"[plan-counts] beta{rc} {dtype}")
    rcb = r * c
    esz = 8 if dtype == torch.float64 else 4
    for name in MATS:
        A = mat(name)
        blocks, values = interval_counts(A, r, c)
        B = spc.csr_to_beta(r, c, A.rowptr, A.colidx, torch.from_numpy(A.values).to(dtype), A.n_cols)
        max0 = 127 if r == 1 else 128 // r
        for kq in (2, 4, 6, 8):
            cap = (64 * kq - 1) * (16 // esz)
            want0 = replay(blocks, np.zeros_like(values), cap // rcb, 1 << 40, max0)
            info = B.plan(0, 0, 0, kq).info()
            assert (info["n_tiles"], info["n_long"]) == want0, (name, "mode 0", kq)
            nbx = min(4032 // rcb, 128 * kq // r - 64 // rcb + 1)
            want3 = replay(blocks, values, nbx, cap, max0)
            modes = (3, 4) if rc == (1, 8) else (3,)
            for m in modes:
                info = B.plan(0, 0, m, kq).info()
                assert (info["n_tiles"], info["n_long"]) == want3, (name, f"mode {m}", kq)
        for tb in (1024, 2048, 3072, 4032):
            want1 = replay(blocks, np.zeros_like(values), tb // rcb, 1 << 40, 256 // r)
            info = B.plan(tb, 0, 1, 0).info()
            assert (info["n_tiles"], info["n_long"]) == want1, (name, "mode 1", tb)
