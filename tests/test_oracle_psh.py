"""Pins of the oracle's perfect spatial hash (Eq. 1)."""
from math import gcd

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def levels(tiny, tiny_keys):
    return [oracle.build_psh_level(k, N, seed=1) for N, k in zip(tiny.res, tiny_keys)]


def test_sizes_follow_rules(tiny, tiny_keys, levels):
    for N, k, L in zip(tiny.res, tiny_keys, levels):
        n = len(k)
        assert 80 * L.mbar ** 3 >= 100 * n > 80 * (L.mbar - 1) ** 3
        assert gcd(L.mbar, L.rbar) == 1 and L.mbar * L.rbar >= N + 1 and 2 * L.rbar ** 3 >= n
        assert 2 <= L.rbar <= 1024 and 1024 * L.mbar >= N + 1
        assert L.phi.shape == (L.rbar ** 3,)
        off = np.stack([L.phi & 1023, (L.phi >> 10) & 1023, (L.phi >> 20) & 1023], 1)
        assert off.max() < L.mbar and (L.phi >> 30).max() == 0


def test_injective_by_brute_force(tiny_keys, levels):
    for k, L in zip(tiny_keys, levels):
        s = L.slots.tolist()
        assert len(set(s)) == len(s)
        assert min(s) >= 0 and max(s) < L.mbar ** 3


def test_lookup_equals_dictionary(tiny, tiny_keys, levels):
    for l, (N, k, L) in enumerate(zip(tiny.res, tiny_keys, levels)):
        feats = synth.table_features(2, l, k, N)
        table = np.zeros((L.mbar ** 3, 2), np.float32)
        table[L.slots] = feats
        d = dict(zip(map(tuple, k.tolist()), feats))
        got = table[oracle.psh_slots(L, k)]
        want = np.array([d[tuple(v)] for v in k.tolist()])
        assert np.array_equal(got, want)
        assert np.array_equal(oracle.psh_slots(L, k), L.slots)


def test_bucket_members_differ_mod_mbar(tiny_keys, levels):
    for k, L in zip(tiny_keys, levels):
        q = k % L.rbar
        ql = (q[:, 2] * L.rbar + q[:, 1]) * L.rbar + q[:, 0]
        h = k % L.mbar
        hl = (h[:, 2] * L.mbar + h[:, 1]) * L.mbar + h[:, 0]
        pairs = set(zip(ql.tolist(), hl.tolist()))
        assert len(pairs) == len(k)


def test_reproducible_and_seed_dependent(tiny, tiny_keys, levels):
    again = oracle.build_psh_level(tiny_keys[1], tiny.res[1], seed=1)
    assert np.array_equal(again.phi, levels[1].phi) and np.array_equal(again.slots, levels[1].slots)
    other = oracle.build_psh_level(tiny_keys[1], tiny.res[1], seed=99)
    assert len(set(other.slots.tolist())) == len(other.slots)


def test_neighbouring_keys_get_neighbouring_slots(tiny_keys, levels):
    # the construction favours equal offsets in neighbouring buckets, which puts
    # x-neighbours in consecutive slots (the coherence claimed in Sec. 4.1)
    for k, L in zip(tiny_keys, levels):
        d = dict(zip(map(tuple, k.tolist()), L.slots.tolist()))
        pairs = [(d[v], d[(v[0] + 1, v[1], v[2])]) for v in d if (v[0] + 1, v[1], v[2]) in d]
        adj = np.mean([b == a + 1 for a, b in pairs])
        assert adj > 0.5, adj


def test_tiny_hand_case():
    # 8 keys of one cell, N = 1, full table: mbar = 2, rbar = 1 -> 3 (gcd 1)
    k = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)])
    L = oracle.build_psh_level(k, 1, seed=1, load_pct=100, bucket_keys=6)
    assert L.mbar == 2 and L.rbar == 3
    assert sorted(L.slots.tolist()) == list(range(8))
    # one bucket per key and a neighbour-first search: the first bucket takes
    # the first pseudo-random offset, every later bucket copies a placed
    # neighbour's, so all keys share one offset and x-neighbours are adjacent
    L = oracle.build_psh_level(k, 1, seed=1, load_pct=100, bucket_keys=1)
    assert L.mbar == 2 and L.rbar == 3
    used = L.phi[[(z * 3 + y) * 3 + x for x, y, z in k.tolist()]]
    assert len(set(used.tolist())) == 1
    r = oracle.psh.splitmix64(oracle.psh.splitmix64(1))
    assert int(used[0]) == (r % 2) | (((r >> 21) % 2) << 10) | (((r >> 42) % 2) << 20)
    s = L.slots.tolist()
    assert all(s[i + 1] == s[i] + 1 for i in range(0, 8, 2))


def test_sizes_at_large_resolution_with_few_keys():
    # one key at N = 4000: mbar is raised so that rbar stays <= 1024
    L = oracle.build_psh_level(np.array([[3999, 0, 17]]), 4000, seed=1)
    assert L.mbar == 4 and L.rbar <= 1024 and L.mbar * L.rbar >= 4001
    assert L.slots.tolist() == oracle.psh_slots(L, [[3999, 0, 17]]).tolist()


def test_splitmix64_published_vector():
    # first output of SplitMix64 seeded with 0 (Steele, Lea & Flood 2014;
    # the reference vector quoted with Vigna's C implementation)
    assert oracle.psh.splitmix64(0) == 0xE220A8397B1DCDAF
