"""Fiat-Shamir transcript (oracle; test infrastructure).

The paper makes its interactive protocols non-interactive by deriving every
verifier challenge from a hash of all earlier public messages (footnote to the
zkSwiGLU activation check in Sec. IV-A; random-oracle model in Sec. V).  It
does not fix the hash or the byte layout, so this project fixes them:

  init:     st = H(DOMAIN || u64 seed || u32 group_id || u32 n_products
                   || (u32 D0, u32 D1, u32 D2) for each product)
  absorb:   st = H(st || label || data)
  squeeze:  for ctr = 0, 1, ...:  h = H(st || label || u32 ctr);
            x = int_le(h) mod 2^255;  if x < p: st = h, return x

H is SHA-256 (FIPS 180-4, here hashlib's); integers are little-endian; field
elements are 32-byte canonical little-endian strings.  Rejection sampling
keeps the challenge exactly uniform on [0, p).
"""
import hashlib
import struct

from .field import P

DOMAIN = b"VeriLoRA-zkMat-v1"
MASK255 = (1 << 255) - 1


def sha256(data: bytes) -> bytes:
    return hashlib.sha256(data).digest()


class Transcript:
    def __init__(self, seed: int, group_id: int, shapes):
        msg = DOMAIN + struct.pack("<QII", seed, group_id, len(shapes))
        for (d0, d1, d2) in shapes:
            msg += struct.pack("<III", d0, d1, d2)
        self.state = sha256(msg)

    @classmethod
    def from_state(cls, state: bytes) -> "Transcript":
        """A transcript that continues from a given 32-byte state."""
        t = cls.__new__(cls)
        t.state = bytes(state)
        return t

    def fork(self, label: bytes, k: int) -> "Transcript":
        """An independent branch: a new transcript whose state is
        H(st || label || u32 k); this transcript is left unchanged."""
        return Transcript.from_state(sha256(self.state + label + struct.pack("<I", k)))

    def absorb(self, label: bytes, data: bytes) -> None:
        self.state = sha256(self.state + label + data)

    def squeeze(self, label: bytes) -> int:
        ctr = 0
        while True:
            h = sha256(self.state + label + struct.pack("<I", ctr))
            x = int.from_bytes(h, "little") & MASK255
            if x < P:
                self.state = h
                return x
            ctr += 1
