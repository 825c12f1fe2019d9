"""The prime field F used for every proof (oracle; test infrastructure).

The paper asks for a field of about 2^254 elements "such as" the one from
BLS12-381 (Sec. V, security model).  This project fixes F to the BLS12-381
scalar field: p = x^4 - x^2 + 1 for the curve parameter x = -0xd201000000010000.

Elements are Python ints in [0, p).  Their byte encoding is the canonical value
as 32 bytes, little-endian; a decoder rejects non-canonical strings (>= p).
Signed integers enter the field as x mod p, so a negative x becomes p - |x|.
"""
P = 0x73eda753299d7d483339d80809a1d80553bda402fffe5bfeffffffff00000001
ELEM_BYTES = 32


def lift(x) -> int:
    """Signed integer -> field element (negatives map to p - |x|)."""
    return int(x) % P


def enc(x: int) -> bytes:
    if not 0 <= x < P:
        raise ValueError("not a canonical field element")
    return int(x).to_bytes(ELEM_BYTES, "little")


def dec(b: bytes) -> int:
    if len(b) != ELEM_BYTES:
        raise ValueError("field element must be 32 bytes")
    x = int.from_bytes(b, "little")
    if x >= P:
        raise ValueError("non-canonical field element")
    return x


def inv(x: int) -> int:
    """Multiplicative inverse (Python's modular inverse, by the extended
    Euclidean algorithm; equal to x^(p-2) by Fermat's little theorem)."""
    if x % P == 0:
        raise ZeroDivisionError("0 has no inverse")
    return pow(x, -1, P)
