"""Pins for the oracle's Philox4x32-10: the published known-answer vectors
(Salmon et al., SC 2011; the Random123 distribution's test vectors) and the
exact integer-to-double mapping onto [-1, 1)."""

import numpy as np

KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 0xFFFFFFFF),
     (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_known_answer_vectors(oracle_mod):
    for ctr, key, want in KAT:
        out = oracle_mod.philox4x32_10(*[np.array([c], dtype=np.uint32) for c in ctr], *key)
        assert tuple(int(o[0]) for o in out) == want


def test_random_block_mapping(oracle_mod):
    seed = (7 << 32) | 12345
    n = 1000
    blk = oracle_mod.random_block(seed, n, [0, 5, 2 ** 31])
    assert blk.shape == (n, 3)
    assert blk.min() >= -1.0 and blk.max() < 1.0
    assert abs(blk.mean()) < 0.1
    # recompute three entries with Python integers from the round function
    for r, qi, q in [(0, 0, 0), (999, 1, 5), (517, 2, 2 ** 31)]:
        w = oracle_mod.philox4x32_10(np.array([r], np.uint32), np.array([0], np.uint32),
                                     np.array([q], np.uint32), np.array([0], np.uint32),
                                     seed & 0xFFFFFFFF, seed >> 32)
        u = ((int(w[1][0]) << 32) | int(w[0][0])) >> 11
        assert blk[r, qi] == u * 2.0 ** -52 - 1.0
        assert u < 2 ** 53
