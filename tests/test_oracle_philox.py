"""Pins of the oracle's Philox4x32-10 against the known-answer vectors
published with the generator (Salmon, Moraes, Dror & Shaw, SC 2011; the
Random123 distribution's kat_vectors), and of its conversions."""
import numpy as np
import pytest

from oracle import philox

KAT = [  # (counter, key, output)
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff, 0xffffffff), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,expected", KAT)
def test_known_answers(ctr, key, expected):
    assert philox.philox4x32_10(ctr, key) == expected


def test_uniforms_and_normals():
    u = philox.fill(1234, 7, 3, 20001, normal=False)
    assert (u > 0).all() and (u < 1).all()
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1 / 12) < 0.003
    z = philox.fill(1234, 8, 3, 20000, normal=True)
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1) < 0.02
    # counter-based: number i does not depend on how many are drawn
    np.testing.assert_array_equal(philox.fill(99, 1, 5, 7, True), philox.fill(99, 1, 5, 8, True)[:7])


def test_chain_normal_layout():
    z = philox.chain_normals(5, 3, 42, 1, 9)
    flat = philox.fill(42, 1, 9, 18, normal=True)     # 3 blocks per chain, 6 normals each
    for c in range(3):
        np.testing.assert_array_equal(z[c], flat[6 * c:6 * c + 5])
