"""Pins of the oracle's random number generator (Sec. 3.2, Fig. "rand").

The oracle evaluates each generator step as the integer product a*s mod m.
These tests pin it to things other than itself:
  * the paper's own float-only Schrage evaluation (its figure), emulated
    literally in numpy float32 for EVERY state of every component;
  * number theory: each modulus is prime and each multiplier a primitive
    root, so every component has full period m-1;
  * the output formula against an exact rational evaluation of
    frac(s0/m0 - s1/m1 + s2/m2 - s3/m3) on the *advanced* state;
  * statistical uniformity (the paper's caveat on quality);
  * stream seeding: the two published generators it is built from
    (splitmix64 and Marsaglia's xor128) against their published known
    answers, and the seeding rule composed from those two pinned pieces.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

# constants printed in the paper's figure
Q = (1225, 1585, 2457, 2098)
R = (1112, 367, 92, 265)
A = (3423, 2646, 1707, 1999)
M = (4194287, 4194277, 4194191, 4194167)


def _glsl_float_step(state: np.ndarray, j: int) -> np.ndarray:
    """The figure's float32 step, operation by operation (GLSL mod/sign/floor)."""
    f = np.float32
    s = state.astype(np.float32)
    q, r, a, m = f(Q[j]), f(R[j]), f(A[j]), f(M[j])
    beta = np.floor(s / q)
    modv = s - q * np.floor(s / q)
    p = a * modv - beta * r
    beta = (np.sign(-p) + f(1)) * f(0.5) * m
    return (p + beta).astype(np.float32)


@pytest.mark.parametrize("j", [0, 1, 2, 3])
def test_integer_step_equals_paper_float_step_exhaustively(oracle_lib, j):
    states = np.arange(1, M[j], dtype=np.uint32)
    ours = oracle_lib.rng_step_component(j, states)
    paper = _glsl_float_step(states, j)
    assert np.all(paper == ours.astype(np.float32))
    assert ours.min() >= 1 and ours.max() <= M[j] - 1


def _is_prime(n: int) -> bool:
    if n < 2:
        return False
    i = 2
    while i * i <= n:
        if n % i == 0:
            return False
        i += 1
    return True


def _prime_factors(n: int):
    f, i = set(), 2
    while i * i <= n:
        while n % i == 0:
            f.add(i)
            n //= i
        i += 1
    if n > 1:
        f.add(n)
    return f


@pytest.mark.parametrize("j", [0, 1, 2, 3])
def test_constants_give_full_period(oracle_lib, j):
    # read the multiplier and modulus back from the oracle's behaviour
    a = int(oracle_lib.rng_step_component(j, np.array([1], np.uint32))[0])
    m_minus_a = int(oracle_lib.rng_step_component(j, np.array([M[j] - 1], np.uint32))[0])
    assert a == A[j] and m_minus_a == M[j] - A[j]
    assert _is_prime(M[j])
    # Schrage's conditions used by the float version: q = m div a, r = m mod a, r < q
    assert Q[j] == M[j] // A[j] and R[j] == M[j] % A[j] and R[j] < Q[j]
    for f in _prime_factors(M[j] - 1):
        assert pow(A[j], (M[j] - 1) // f, M[j]) != 1


def test_output_is_fractional_weighted_sum_of_advanced_state(oracle_lib):
    rng = np.random.default_rng(0)
    checked = 0
    for i in range(3000):
        s = np.array([rng.integers(1, M[j]) for j in range(4)], np.uint32)
        u = float(oracle_lib.rng_draw(s, 1)[0])
        adv = [(A[j] * int(s[j])) % M[j] for j in range(4)]
        x = Fraction(adv[0], M[0]) - Fraction(adv[1], M[1]) + Fraction(adv[2], M[2]) - Fraction(adv[3], M[3])
        fr = x - (x.numerator // x.denominator)
        fr = float(fr)
        if min(fr, 1 - fr) < 1e-5:
            continue  # the wrap point: rounding may land on either side
        assert abs(u - fr) <= 4 * 2.0 ** -24, (s, u, fr)
        # and not the unadvanced state's value
        x0 = sum(Fraction(int(s[j]), M[j]) * (1 if j % 2 == 0 else -1) for j in range(4))
        f0 = float(x0 - (x0.numerator // x0.denominator))
        if abs(f0 - fr) > 1e-3:
            assert abs(u - f0) > 1e-4
        checked += 1
    assert checked > 2900


def test_output_range_and_uniformity(oracle_lib):
    u = oracle_lib.rng_streams(seed=11, kind=2, k=0, index0=0, n_streams=2000, n_draws=500).ravel()
    assert u.min() >= 0.0 and u.max() < 1.0
    counts, _ = np.histogram(u, bins=256, range=(0, 1))
    assert stats.chisquare(counts).pvalue > 1e-4
    assert stats.kstest(u.astype(np.float64), "uniform").pvalue > 1e-4
    # serial pairs within a stream
    v = oracle_lib.rng_streams(seed=12, kind=2, k=0, index0=0, n_streams=1000, n_draws=1000)
    a, b = v[:, :-1].ravel(), v[:, 1:].ravel()
    h2, _, _ = np.histogram2d(a, b, bins=16, range=[[0, 1], [0, 1]])
    assert stats.chisquare(h2.ravel()).pvalue > 1e-4
    assert abs(np.corrcoef(a, b)[0, 1]) < 5e-3
    # first draws across neighbouring streams
    first = v[:, 0]
    assert abs(np.corrcoef(first[:-1], first[1:])[0, 1]) < 0.1


def test_stream_seeding_invariants(oracle_lib):
    seen = set()
    for idx in range(20000):
        s = oracle_lib.rng_seed(5, 2, 3, idx)
        assert all(1 <= int(s[j]) <= M[j] - 1 for j in range(4))
        seen.add(tuple(int(x) for x in s))
    assert len(seen) == 20000
    base = tuple(oracle_lib.rng_seed(5, 2, 3, 7))
    for key in [(6, 2, 3, 7), (5, 1, 3, 7), (5, 2, 4, 7), (5, 2, 3, 8), (5, 2, 3, 7 + (1 << 40))]:
        assert tuple(oracle_lib.rng_seed(*key)) != base
    assert tuple(oracle_lib.rng_seed(5, 2, 3, 7)) == base


def test_streams_are_random_access(oracle_lib):
    full = oracle_lib.rng_streams(3, 1, 2, 0, 64, 10)
    part = oracle_lib.rng_streams(3, 1, 2, 40, 4, 10)
    assert np.array_equal(full[40:44], part)


# splitmix64 (Steele, Lea and Flood 2014; Vigna's reference implementation):
# the first outputs from state 0 and from state 1234567 are published test
# values of the generator.
SPLITMIX64_FROM_0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
SPLITMIX64_FROM_1234567 = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                           4593380528125082431, 16408922859458223821]
# Marsaglia (2003), "Xorshift RNGs": xor128 with its published default seed
# x, y, z, w = 123456789, 362436069, 521288629, 88675123.
XOR128_SEED = [123456789, 362436069, 521288629, 88675123]
XOR128_OUT = [3701687786, 458299110, 2500872618, 3633119408, 516391518]


def test_splitmix64_known_answers(oracle_lib):
    assert [int(x) for x in oracle_lib.splitmix64(0, 4)] == SPLITMIX64_FROM_0
    assert [int(x) for x in oracle_lib.splitmix64(1234567, 5)] == SPLITMIX64_FROM_1234567


def test_xor128_known_answers(oracle_lib):
    assert [int(x) for x in oracle_lib.xor128(XOR128_SEED, 5)] == XOR128_OUT


def _seed_from_pinned_parts(oracle_lib, seed, kind, k, index):
    """The stream-seeding rule, composed from the two pinned generators:
    h1 = splitmix64(seed); h2 = splitmix64(h1 ^ (kind << 32 | k));
    w01, w23 = the two splitmix64 outputs from state h2 ^ index; xor128 seeded
    with their 32-bit halves (low first); s_j = 1 + (output 9 + j) mod (m_j - 1)."""
    mask = (1 << 64) - 1
    h1 = int(oracle_lib.splitmix64(seed, 1)[0])
    h2 = int(oracle_lib.splitmix64(h1 ^ ((kind << 32) | k), 1)[0])
    w01, w23 = (int(x) for x in oracle_lib.splitmix64((h2 ^ index) & mask, 2))
    words = [w01 & 0xFFFFFFFF, w01 >> 32, w23 & 0xFFFFFFFF, w23 >> 32]
    if not any(words):
        words[0] = 1
    out = [int(x) for x in oracle_lib.xor128(words, 12)]
    return [1 + out[8 + j] % (M[j] - 1) for j in range(4)]


def test_stream_seeding_is_the_composition_of_the_pinned_generators(oracle_lib):
    keys = [(0, 1, 0, 0), (1, 2, 0, 5), (5, 2, 3, 7), (2 ** 63 + 11, 1, 63, 2 ** 40 + 3),
            (3, 3, 7, 123456), (2 ** 64 - 1, 2, 2 ** 32 - 1, 2 ** 64 - 1)]
    rng = np.random.default_rng(7)
    keys += [(int(rng.integers(0, 2 ** 63)), int(rng.integers(1, 4)), int(rng.integers(0, 64)),
              int(rng.integers(0, 2 ** 40))) for _ in range(200)]
    for key in keys:
        assert [int(x) for x in oracle_lib.rng_seed(*key)] == _seed_from_pinned_parts(oracle_lib, *key), key
