"""Fiat-Shamir challenge from a transcript (test oracle only).

Parallel Accumulation derives its challenges with random oracles (rho_acc,
rho_NARK) that the paper does not instantiate.  Here they are read as a
hash to the field: the 512-bit little-endian integer formed by
SHA-256(0x00 || data) followed by SHA-256(0x01 || data), reduced mod r (two
digests, so the reduction's bias is below 2^-250).  SHA-256 is the standard
library's.

Parity unpinned: the paper fixes no instantiation of these oracles, so no
value outside this build pins the composition; the tests pin only the
SHA-256 it calls (FIPS 180-4 example digests) and the challenge's range.
"""
import hashlib

from .field import R


def challenge(data: bytes) -> int:
    h = hashlib.sha256(b"\x00" + data).digest() + hashlib.sha256(b"\x01" + data).digest()
    return int.from_bytes(h, "little") % R
