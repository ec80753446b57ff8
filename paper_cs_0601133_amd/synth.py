"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  This module holds no arithmetic of the method: it only draws numbers.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  Stream element i of seed s is
mix(s + (i + 1) * 0x9E3779B97F4A7C15) with the published mixing function.
A draw x in [0, 2^64) becomes a value in [0, R) by the multiply-shift map
floor(x * R / 2^64) (bias at most R / 2^64).

Seeds follow one convention: 0x5EED0000 + 1000 * config + tensor, with
tensor 1 = A, 2 = B, 3 = C; serving request r uses 0x5EED5000000 + 16 * r +
tensor.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK32 = np.uint64(0xFFFFFFFF)
_CHUNK = 1 << 22


def seed_for(config, tensor):
    return 0x5EED0000 + 1000 * int(config) + int(tensor)


def request_seed(req, tensor):
    return 0x5EED5000000 + 16 * int(req) + int(tensor)


def splitmix64(seed, count, start=0):
    """count consecutive outputs of the SplitMix64 stream of ``seed``."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _below(x, R):
    """floor(x * R / 2^64) for uint64 x and 0 < R < 2^32, without overflow."""
    R = np.uint64(R)
    hi = x >> np.uint64(32)
    lo = x & _MASK32
    with np.errstate(over="ignore"):
        t = hi * R + ((lo * R) >> np.uint64(32))
    return t >> np.uint64(32)


def uniform_below(seed, shape, R):
    """uint32 array of the given shape, entries uniform in [0, R)."""
    if not (0 < R < (1 << 32)):
        raise ValueError("range must be in (0, 2^32)")
    count = int(np.prod(shape)) if len(shape) else 1
    out = np.empty(count, dtype=np.uint32)
    for s in range(0, count, _CHUNK):
        e = min(count, s + _CHUNK)
        out[s:e] = _below(splitmix64(seed, e - s, s), R).astype(np.uint32)
    return out.reshape(shape)


def residues(seed, shape, p):
    """Residues uniform in [0, p)."""
    return uniform_below(seed, shape, p)


def signed_ints(seed, shape, bound):
    """int64 entries uniform in [-bound, bound]."""
    u = uniform_below(seed, shape, 2 * int(bound) + 1).astype(np.int64)
    return u - int(bound)


def is_prime(n):
    """Deterministic Miller-Rabin for n < 2^64 (fixed witness set)."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for q in small:
        if n % q == 0:
            return n == q
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def primes_below(limit, count):
    """The ``count`` largest primes below ``limit``, in decreasing order."""
    out = []
    q = limit - 1
    while len(out) < count and q >= 2:
        if is_prime(q):
            out.append(q)
        q -= 1
    return out
