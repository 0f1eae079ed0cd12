"""Fiat-Shamir challenge from a transcript (test oracle only).

Parallel Accumulation derives its challenges with random oracles (rho_acc,
rho_NARK) that the paper does not instantiate.  Here they are read as a
hash to the field: the 512-bit little-endian integer formed by
SHA-256(0x00 || data) followed by SHA-256(0x01 || data), reduced mod r (two
digests, so the reduction's bias is below 2^-250).  SHA-256 is the standard
library's.
"""
import hashlib

from .field import R


def challenge(data: bytes) -> int:
    h = hashlib.sha256(b"\x00" + data).digest() + hashlib.sha256(b"\x01" + data).digest()
    return int.from_bytes(h, "little") % R
