"""The rule by which the GPU walks find the clock of a round of SSA attempts
without adding the waiting times one by one, checked on the CPU against
binary64 addition itself (Python floats are IEEE binary64 with
round-to-nearest-even).

While the running clock s stays in one binade [2^e, 2^(e+1)), every partial
sum is an integer multiple of h = 2^(e-52), and s + tau rounds to
(s/h + rn(tau/h)) h; so integer prefix sums give every partial sum up to the
first attempt that reaches 2^(e+1) or whose tau/h lies exactly half-way
between two integers (a tie, decided by the parity of the running sum). That
attempt is added as binary64 adds it and the scan resumes in the new binade.
The first attempt whose sum is not below 1 ends the round. These tests check
that this rule, written out here in exact integer arithmetic, gives the same
number of attempts and the same clock, bit for bit, as the serial sum, on
random rounds and on rounds built to hit ties and binade ends.
"""
import math
import random
import struct

import pytest


def serial(clock, taus):
    """Attempts that fire and the clock after them, adding one by one."""
    s, k = clock, 0
    for t in taus:
        s2 = s + t
        if not s2 < 1.0:
            break
        s, k = s2, k + 1
    return k, s


def by_scan(clock, taus):
    """The rule of the GPU walks, with Python integers for the prefix sums."""
    done, s, n = 0, clock, len(taus)
    while done < n:
        if s == 0.0:  # 0 + tau is tau
            if not taus[done] < 1.0:
                break
            s, done = taus[done], done + 1
            continue
        m, e2 = math.frexp(s)          # s = m 2^e2, m in [0.5, 1)
        e = e2 - 1                     # binade [2^e, 2^(e+1))
        h = math.ldexp(1.0, e - 52)
        S0 = int(s / h)                # exact: s is a multiple of h in [2^52, 2^53)
        assert S0 * h == s and 2 ** 52 <= S0 < 2 ** 53
        T = 2 ** 53 - S0
        run, special = 0, n
        for a in range(done, n):
            v = taus[a] / h            # exact: scaling by a power of two
            if math.isinf(v):          # lambda = 0: past any binade end
                special = a
                break
            fl = math.floor(v)
            fr = v - fl
            if fr == 0.5:
                special = a
                break
            run += fl + (1 if fr > 0.5 else 0)
            if run >= T:
                special = a
                break
        # partial sum before `special`, exact
        before = s
        if special > done:
            tot = 0
            for a in range(done, special):
                v = taus[a] / h
                fl = math.floor(v)
                tot += fl + (1 if v - fl > 0.5 else 0)
            before = (S0 + tot) * h
        if special == n:
            return n, before
        s2 = before + taus[special]    # the attempt binary64 adds itself
        if not s2 < 1.0:
            return special, before
        s, done = s2, special + 1
    return done, s


def bits(x):
    return struct.unpack("<q", struct.pack("<d", x))[0]


def check(clock, taus):
    a = serial(clock, taus)
    b = by_scan(clock, taus)
    assert a[0] == b[0] and bits(a[1]) == bits(b[1]), (clock, a, b)
    return a


@pytest.mark.parametrize("seed", range(8))
def test_random_rounds(seed):
    rng = random.Random(seed)
    for _ in range(400):
        lam = 10 ** rng.uniform(0, 6)            # rates from 1 to 10^6 per day
        clock = rng.choice([0.0, rng.random() * rng.choice([1e-6, 1e-3, 0.1, 1.0])])
        taus = [-math.log(1.0 - rng.random()) / lam for _ in range(rng.choice([64, 256]))]
        check(clock, taus)


def test_rounds_crossing_many_binades_from_zero():
    rng = random.Random(11)
    for _ in range(200):
        lam = 10 ** rng.uniform(1, 5)
        taus = [-math.log(1.0 - rng.random()) / lam for _ in range(256)]
        k, s = check(0.0, taus)
        assert k == 256 or s < 1.0


def test_constructed_ties():
    # waiting times exactly half a spacing above a multiple: round to even
    # decides, which depends on the running sum's parity
    rng = random.Random(12)
    for _ in range(300):
        e = rng.randint(-12, -1)
        h = math.ldexp(1.0, e - 52)
        clock = (2 ** 52 + rng.randint(0, 2 ** 52 - 1)) * h      # in [2^e, 2^(e+1))
        taus = []
        for _ in range(64):
            if rng.random() < 0.3:
                taus.append((rng.randint(1, 2 ** 20) + 0.5) * h)  # a tie
            else:
                taus.append(rng.randint(1, 2 ** 30) * h * rng.random())
        check(clock, taus)


def test_constructed_binade_ends_and_window_end():
    # partial sums that land exactly on 2^(e+1), and on 1.0 (not below 1)
    for e in (-5, -2, -1):
        h = math.ldexp(1.0, e - 52)
        start = math.ldexp(1.0, e + 1) - 3 * h
        check(start, [h, h, h, h, h])
        check(start, [1.5 * h, 1.5 * h, h])
    check(1.0 - math.ldexp(1.0, -53), [math.ldexp(1.0, -54)])      # tie at 1: rounds to 1.0, does not fire
    check(0.5, [0.25, 0.125, 0.125, 0.0625])


def test_zero_rate_attempt_never_fires():
    k, s = check(0.25, [0.1, math.inf, 0.1])
    assert k == 1
