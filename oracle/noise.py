"""Static noise draws of Eq. 1 (parameter = baseline + stochastic part),
written for checking the library's own draws.  Test infrastructure only:
nothing in the product path imports this module.

Counter-based generator: Philox4x32-10 from its definition in Salmon,
Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
(SC 2011): a 128-bit counter of four 32-bit words and a 64-bit key of two;
ten rounds, each multiplying words 0 and 2 by fixed constants and mixing
the high halves of the products with words 1 and 3 and the key, the key
advancing by fixed Weyl increments between rounds.  Pinned by the
generator's published known-answer vectors (tests/golden).

Mapping used by the library (include/ctqw.h, ctqw_draw_params): one block
per parameter, counter (index, kind, r mod 2^32, r div 2^32) with kind 0
for bonds, 1 for sites, 2 for the interaction, key (seed mod 2^32,
seed div 2^32); u, v are 53-bit fractions from (w0, w1) and (w2, w3);
uniform a + (b - a) u, normal a + b sqrt(-2 log(1 - u)) cos(2 pi v)
(Box and Muller, 1958).
"""

from __future__ import annotations

import math

MASK32 = 0xFFFFFFFF
# round multipliers and key increments of Philox4x32 (Salmon et al., Sec. 5)
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85

BOND, SITE, INTERACTION = 0, 1, 2


def philox4x32(counter, key, rounds: int = 10):
    """One Philox4x32 block: counter = 4 words, key = 2 words."""
    x = [int(c) & MASK32 for c in counter]
    k = [int(c) & MASK32 for c in key]
    for rnd in range(rounds):
        if rnd:
            k = [(k[0] + PHILOX_W0) & MASK32, (k[1] + PHILOX_W1) & MASK32]
        prod0 = PHILOX_M0 * x[0]
        prod1 = PHILOX_M1 * x[2]
        hi0, lo0 = prod0 >> 32, prod0 & MASK32
        hi1, lo1 = prod1 >> 32, prod1 & MASK32
        x = [hi1 ^ x[1] ^ k[0], lo1, hi0 ^ x[3] ^ k[1], lo0]
    return x


def unit53(hi: int, lo: int) -> float:
    """53-bit fraction in [0, 1): the top 27 bits of hi, then 26 of lo."""
    return ((hi >> 5) * 67108864 + (lo >> 6)) / 9007199254740992.0


def draw(dist: str, a: float, b: float, seed: int, r: int, kind: int, index: int) -> float:
    """The stochastic part of one parameter."""
    if dist == "none":
        return 0.0
    w = philox4x32([index, kind, r & MASK32, r >> 32], [seed & MASK32, seed >> 32])
    u = unit53(w[0], w[1])
    if dist == "uniform":
        return a + (b - a) * u
    if dist == "normal":
        v = unit53(w[2], w[3])
        return a + b * (math.sqrt(-2.0 * math.log(1.0 - u)) * math.cos(6.283185307179586 * v))
    raise ValueError(dist)


def draw_params(Ns, periodic: bool, *, J_base=None, eps_base=None, U_base: float = 0.0,
                J_noise=None, eps_noise=None, U_noise=None, seed: int = 0):
    """Packed (J, eps, U) lists for realisations of sizes Ns, with the
    library's conventions (J_base None -> 1, eps_base None -> 0)."""
    none = ("none", 0.0, 0.0)
    jn, en, un = J_noise or none, eps_noise or none, U_noise or none
    J, eps, U = [], [], []
    for r, N in enumerate(Ns):
        nb = N if periodic else N - 1
        for i in range(nb):
            J.append((1.0 if J_base is None else float(J_base[i])) + draw(*jn, seed, r, BOND, i))
        for i in range(N):
            eps.append((0.0 if eps_base is None else float(eps_base[i])) + draw(*en, seed, r, SITE, i))
        U.append(float(U_base) + draw(*un, seed, r, INTERACTION, 0))
    return J, eps, U
