"""The arithmetic behind the modular split, checked on the CPU with Python integers (no GPU, no
library): the moduli the library uses, and the identity that lets it form each complex product
modulo p from two real ones.

For odd p whose prime factors are all 1 mod 4, -1 has a square root j mod p, and the map
x = a + ib -> (a + j b, a - j b) mod p turns sums and products of Gaussian integers mod p into
componentwise sums and products.  The contraction therefore forms z1 = sum (Xr - j Xi)(Yr + j Yi)
and z2 = sum (Xr + j Xi)(Yr - j Yi) mod p and recovers Re conj(X)^T Y = (z1 + z2) / 2 and
Im = (z1 - z2) / (2 j) mod p; the Chinese remainder theorem then rebuilds the exact integers from
the residues of all moduli."""
import math

import numpy as np

# the moduli as include/flapw.h lists them (FLAPW_PREC_SPLIT_I8_MOD), in the library's order
MODULI = [241, 233, 229, 221, 205, 197, 193, 181, 173, 157, 149, 137, 113, 109]


def _sqrt_minus_one(p):
    return next((x for x in range(1, p) if (x * x + 1) % p == 0), 0)


def _sym(a, p):
    r = a % p
    return r - p if r > p // 2 else r


def test_moduli_are_the_greedy_set_of_odd_coprime_numbers_with_a_square_root_of_minus_one():
    chosen, c = [], 255
    while len(chosen) < 14:
        if _sqrt_minus_one(c) and all(math.gcd(c, m) == 1 for m in chosen):
            chosen.append(c)
        c -= 2
    assert chosen == MODULI
    # every prime factor of every modulus is 1 mod 4 (the condition for -1 to be a square)
    for p in MODULI:
        q, f = p, 2
        while q > 1:
            while q % f == 0:
                assert f % 4 == 1, (p, f)
                q //= f
            f += 1
    # 241 is the largest odd number <= 255 in which -1 is a square
    assert all(_sqrt_minus_one(c) == 0 for c in range(243, 256, 2))


def test_integer_range_per_count():
    """B = (log2 M - 1)/2 - 0.001 (capped at 50): 10 moduli give B = 37.76, 11 give 41.37."""
    for nm, b in ((10, 37.763), (11, 41.372), (14, 50.0)):
        lg = sum(math.log2(p) for p in MODULI[:nm])
        assert abs(min(50.0, (lg - 1.0) / 2.0 - 0.001) - b) < 1e-3, (nm, lg)


def test_two_real_products_give_the_complex_product():
    rng = np.random.default_rng(1602)
    for p in MODULI:
        j = _sqrt_minus_one(p)
        assert (j * j + 1) % p == 0
        h2, h2j = pow(2, -1, p), pow(2 * j, -1, p)
        for _ in range(20):
            k = int(rng.integers(1, 40))
            xr, xi, yr, yi = (rng.integers(-2 ** 40, 2 ** 40, size=k).tolist() for _ in range(4))
            re = sum(a * c + b * d for a, b, c, d in zip(xr, xi, yr, yi))     # Re conj(x)^T y
            im = sum(a * d - b * c for a, b, c, d in zip(xr, xi, yr, yi))     # Im conj(x)^T y
            # residues as the slicing kernel stores them: symmetric, the left operand conjugated
            u1 = [_sym(_sym(a, p) - j * _sym(b, p), p) for a, b in zip(xr, xi)]
            u2 = [_sym(_sym(a, p) + j * _sym(b, p), p) for a, b in zip(xr, xi)]
            y1 = [_sym(_sym(c, p) + j * _sym(d, p), p) for c, d in zip(yr, yi)]
            y2 = [_sym(_sym(c, p) - j * _sym(d, p), p) for c, d in zip(yr, yi)]
            assert all(abs(v) <= (p - 1) // 2 for v in u1 + u2 + y1 + y2)
            z1 = sum(a * b for a, b in zip(u1, y1))
            z2 = sum(a * b for a, b in zip(u2, y2))
            assert _sym((z1 + z2) * h2, p) == _sym(re, p)
            assert _sym((z1 - z2) * h2j, p) == _sym(im, p)


def test_crt_rebuilds_products_within_the_range():
    """Residues of 11 moduli determine any integer of magnitude below M/2 (here the complex
    products of columns with 2-norm at most 2^B, |C| <= 2^(2B) < M/2 by Cauchy-Schwarz)."""
    rng = np.random.default_rng(7)
    mods = MODULI[:11]
    M = math.prod(mods)
    b = (sum(math.log2(p) for p in mods) - 1.0) / 2.0 - 0.001
    assert 2 ** (2 * b) < M / 2
    for _ in range(200):
        c = int(rng.integers(-2 ** 62, 2 ** 62)) * int(rng.integers(1, 2 ** 20))
        c = max(-(M // 2 - 1), min(M // 2 - 1, c))
        x = 0
        for p in mods:
            w = pow(M // p, -1, p)
            x += (c % p) * w * (M // p)
        x %= M
        if x > M // 2:
            x -= M
        assert x == c
