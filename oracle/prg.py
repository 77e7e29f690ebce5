"""The PRG of the silent offline phase, and the random hint keys it expands -- TEST
INFRASTRUCTURE ONLY (see the package docstring).

ZipPIR lowers its offline communication to a public key and a seed (Sec. 4.3, "Lowering
offline communication costs"): the random ciphertexts ck_r of Alg. 5's Setup are drawn from a
PRG that client and server both run from the seed, and one seed yields the keys of many
queries (Sec. 4.3, "Supporting multiple queries").  The paper does not name the PRG.  This
build takes the ChaCha20 keystream of RFC 8439 with the seed as the 256-bit key, and samples
each ck_r entry uniformly from Z_{N^2} (Alg. 5 samples ck_r from Z_{N^2}^n) by rejection:

* ChaCha20 block (RFC 8439, Sec. 2.3): the 4x4 state of 32-bit words
      constants 0x61707865 0x3320646e 0x79622d32 0x6b206574 | key (8 words, little-endian)
      | block counter | nonce (3 words, little-endian),
  twenty rounds (ten column rounds alternating with ten diagonal rounds) of the quarter round
      a += b; d ^= a; d <<<= 16;  c += d; b ^= c; b <<<= 12;
      a += b; d ^= a; d <<<= 8;   c += d; b ^= c; b <<<= 7,
  then the input state added word by word; the block is the 16 words little-endian.
* Entry k of query q, attempt r: the keystream under nonce (q, k, r) (three little-endian
  words), blocks 0, 1, ... as one little-endian sequence of 32-bit words w_0 w_1 ...; the
  candidate is sum_i w_i 2^(32 i) over W = ceil(bits(N^2) / 32) words, keeping its low
  bits(N^2) bits.  The first candidate below N^2 (attempts r = 0, 1, ...) is ck_r[k].
  A candidate is accepted with probability N^2 / 2^bits(N^2) > 1/2.

Every entry is uniform over [0, N^2); it is a unit of Z_{N^2} except with probability about
2 / sqrt(N), as the paper notes for Alg. 5's sampling.
"""
from __future__ import annotations

MASK = 0xFFFFFFFF
CONSTANTS = (0x61707865, 0x3320646E, 0x79622D32, 0x6B206574)   # "expand 32-byte k"


def _rotl(x: int, n: int) -> int:
    return ((x << n) | (x >> (32 - n))) & MASK


def quarter_round(a: int, b: int, c: int, d: int) -> tuple[int, int, int, int]:
    """RFC 8439, Sec. 2.1."""
    a = (a + b) & MASK
    d = _rotl(d ^ a, 16)
    c = (c + d) & MASK
    b = _rotl(b ^ c, 12)
    a = (a + b) & MASK
    d = _rotl(d ^ a, 8)
    c = (c + d) & MASK
    b = _rotl(b ^ c, 7)
    return a, b, c, d


def _words_le(data: bytes) -> list[int]:
    return [int.from_bytes(data[4 * i:4 * i + 4], "little") for i in range(len(data) // 4)]


def block_words(key: bytes, counter: int, nonce: bytes) -> list[int]:
    """The 16 output words of one ChaCha20 block (RFC 8439, Sec. 2.3)."""
    assert len(key) == 32 and len(nonce) == 12
    init = list(CONSTANTS) + _words_le(key) + [counter & MASK] + _words_le(nonce)
    x = list(init)
    # a column round on (0,4,8,12) (1,5,9,13) (2,6,10,14) (3,7,11,15), then a diagonal round
    # on (0,5,10,15) (1,6,11,12) (2,7,8,13) (3,4,9,14); ten of each
    for _ in range(10):
        for i0, i1, i2, i3 in ((0, 4, 8, 12), (1, 5, 9, 13), (2, 6, 10, 14), (3, 7, 11, 15),
                               (0, 5, 10, 15), (1, 6, 11, 12), (2, 7, 8, 13), (3, 4, 9, 14)):
            x[i0], x[i1], x[i2], x[i3] = quarter_round(x[i0], x[i1], x[i2], x[i3])
    return [(a + b) & MASK for a, b in zip(x, init)]


def block(key: bytes, counter: int, nonce: bytes) -> bytes:
    """One serialized 64-byte ChaCha20 block."""
    return b"".join(w.to_bytes(4, "little") for w in block_words(key, counter, nonce))


def keystream_words(key: bytes, nonce: bytes, nwords: int) -> list[int]:
    """The first nwords 32-bit words of the keystream (blocks 0, 1, ...)."""
    out: list[int] = []
    counter = 0
    while len(out) < nwords:
        out += block_words(key, counter, nonce)
        counter += 1
    return out[:nwords]


def nonce_words(*words: int) -> bytes:
    """Three 32-bit words as a 12-byte little-endian nonce."""
    assert len(words) == 3
    return b"".join((w & MASK).to_bytes(4, "little") for w in words)


def random_key_entry(seed: bytes, N: int, query: int, k: int) -> int:
    """ck_r[k] of query `query`: the first candidate below N^2 (see the module docstring)."""
    N2 = N * N
    bits = N2.bit_length()
    W = (bits + 31) // 32
    r = 0
    while True:
        ws = keystream_words(seed, nonce_words(query, k, r), W)
        cand = sum(w << (32 * i) for i, w in enumerate(ws)) & ((1 << bits) - 1)
        if cand < N2:
            return cand
        r += 1


def random_key(seed: bytes, N: int, n: int, query: int) -> list[int]:
    """The n random ciphertexts ck_r of one query (Alg. 5 Setup, drawn from the seed)."""
    return [random_key_entry(seed, N, query, k) for k in range(n)]
