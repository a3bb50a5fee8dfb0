"""Second, independent transcription of the integer generators in plain Python
integers (test-side only).

It is not itself a pin of the oracle (both are transcriptions of the same
published algorithms); its job is to (a) catch implementation slips in the C++
oracle, such as overflow, shift or index errors, on many random inputs, and
(b) carry a configurable Threefry4x32 mixing schedule so that its shared
machinery (rotations, key schedule, injections) can be checked against
rocRAND, whose Threefry4x32 changes mixing pairs every second round rather
than every round.
"""
from __future__ import annotations

M32 = 0xFFFFFFFF
M64 = 0xFFFFFFFFFFFFFFFF


def rotl(x, r, bits):
    mask = (1 << bits) - 1
    return ((x << r) | (x >> (bits - r))) & mask


# ---- Philox4x32-10 (Salmon et al. SC'11) ---------------------------------
def philox4x32_10(ctr, key):
    x0, x1, x2, x3 = ctr
    k0, k1 = key
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & M32
            k1 = (k1 + 0xBB67AE85) & M32
        p0 = 0xD2511F53 * x0
        p1 = 0xCD9E8D57 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0, p1 & M32, (p0 >> 32) ^ x3 ^ k1, p0 & M32)
    return [x0, x1, x2, x3]


# ---- Threefry4x32 with a selectable mixing schedule ------------------------
ROT4 = [(10, 26), (11, 21), (13, 27), (23, 5), (6, 20), (17, 11), (25, 10), (18, 20)]


def threefry4x32(ctr, key, rounds=20, schedule="every_round"):
    """schedule 'every_round': pairs (0,1)(2,3) on even rounds, (0,3)(2,1) on
    odd rounds (the Threefish word permutation after each round).
    schedule 'every_second_round': pairs switch when bit 1 of the round index
    changes (the schedule rocRAND implements)."""
    ks = list(key) + [0x1BD11BDA ^ key[0] ^ key[1] ^ key[2] ^ key[3]]
    x = [(ctr[i] + ks[i]) & M32 for i in range(4)]
    for r in range(rounds):
        ra, rb = ROT4[r % 8]
        odd = (r & 1) if schedule == "every_round" else ((r >> 1) & 1)
        a, b, c, d = (0, 1, 2, 3) if not odd else (0, 3, 2, 1)
        x[a] = (x[a] + x[b]) & M32
        x[b] = rotl(x[b], ra, 32) ^ x[a]
        x[c] = (x[c] + x[d]) & M32
        x[d] = rotl(x[d], rb, 32) ^ x[c]
        if r % 4 == 3:
            s = (r + 1) // 4
            for i in range(4):
                x[i] = (x[i] + ks[(s + i) % 5]) & M32
            x[3] = (x[3] + s) & M32
    return x


# ---- Threefry2x64-20 --------------------------------------------------------
ROT2 = [16, 42, 12, 31, 16, 32, 24, 21]


def threefry2x64_20(ctr, key):
    ks = [key[0], key[1], 0x1BD11BDAA9FC1A22 ^ key[0] ^ key[1]]
    x0 = (ctr[0] + ks[0]) & M64
    x1 = (ctr[1] + ks[1]) & M64
    for r in range(20):
        x0 = (x0 + x1) & M64
        x1 = rotl(x1, ROT2[r % 8], 64) ^ x0
        if r % 4 == 3:
            s = (r + 1) // 4
            x0 = (x0 + ks[s % 3]) & M64
            x1 = (x1 + ks[(s + 1) % 3] + s) & M64
    return [x0, x1]


# ---- Squares32 (Widynski) and the SplitMix64-based key ---------------------
def squares32(ctr, key):
    y = (ctr * key) & M64
    z = (y + key) & M64
    x = y
    for add in (y, z, y):
        x = (x * x + add) & M64
        x = ((x >> 32) | (x << 32)) & M64
    return ((x * x + z) & M64) >> 32


def squares_key(seed):
    z = (seed + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return (z ^ (z >> 31)) | 1


# ---- Tyche (Neves and Araujo) ---------------------------------------------
def tyche_mix(a, b, c, d):
    a = (a + b) & M32; d = rotl(d ^ a, 16, 32)
    c = (c + d) & M32; b = rotl(b ^ c, 12, 32)
    a = (a + b) & M32; d = rotl(d ^ a, 8, 32)
    c = (c + d) & M32; b = rotl(b ^ c, 7, 32)
    return a, b, c, d


def tyche_outputs(seed, c_xor, d_xor, count):
    st = (seed >> 32, seed & M32, 2654435769 ^ c_xor, 1367130551 ^ d_xor)
    for _ in range(20):
        st = tyche_mix(*st)
    out = []
    for _ in range(count):
        st = tyche_mix(*st)
        out.append(st[1])
    return out


# ---- stream model -----------------------------------------------------------
def word(gen, seed, ctr, p):
    lo, hi = seed & M32, seed >> 32
    b, w = p >> 2, p & 3
    if gen == 0:
        return philox4x32_10([b & M32, ctr, 0, 0], [lo, hi])[w]
    if gen == 1:
        return threefry4x32([b & M32, ctr, 0, 0], [lo, hi, 0, 0])[w]
    if gen == 2:
        x0, x1 = threefry2x64_20([b, ctr], [seed, 0])
        return [x0 & M32, x0 >> 32, x1 & M32, x1 >> 32][w]
    if gen == 3:
        return squares32((ctr << 32) | p, squares_key(seed))
    if gen == 4:
        t, r = divmod(p, 16384)
        lane, k, wi = (r // 4) % 64, r // 256, r % 4
        return tyche_outputs(seed, t * 64 + lane, ctr, 4 * k + wi + 1)[-1]
    raise ValueError(gen)
