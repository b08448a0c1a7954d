"""Readers for the hand-worked fixtures under tests/golden/."""
import os
import struct

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield [p.strip() for p in line.split("|")]


def bits_to_f32(h):
    return struct.unpack("<f", struct.pack("<I", int(h, 16)))[0]


def f32_bits(x):
    return struct.unpack("<I", struct.pack("<f", x))[0]


def select_cases():
    for vals, k, idx, bits in _lines("select_hand.txt"):
        yield ([float(v) for v in vals.split()], int(k), [int(i) for i in idx.split()],
               [int(b, 16) for b in bits.split()])


def lattice_cases():
    for k, node, idx, dist in _lines("lattice_knng.txt"):
        yield int(k), int(node), [int(i) for i in idx.split()], [float(x) for x in dist.split()]


def partition_cases():
    for vals, piv, lanes, L in _lines("partition_example.txt"):
        yield [float(v) for v in vals.split()], float(piv), [int(x) for x in lanes.split()], int(L)
