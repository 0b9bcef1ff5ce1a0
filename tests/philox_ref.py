"""Plain-Python references for the pattern generator's noise (test helpers).

Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011) and the PTRS Poisson sampler (Hormann, "The
transformed rejection method for generating Poisson random variables",
Insurance: Mathematics and Economics 12, 1993), written from their published
definitions; slow, for small checks only.
"""
import math

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & MASK, p1 & MASK, ((p0 >> 32) ^ c3 ^ k1) & MASK, p0 & MASK
        k0 = (k0 + W0) & MASK
        k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def uniforms2(p, attempt, stream, key):
    c = philox4x32_10((p, attempt, stream, 0), key)
    u = ((c[0] >> 5) * 67108864 + (c[1] >> 6)) / 9007199254740992.0
    v = ((c[2] >> 5) * 67108864 + (c[3] >> 6)) / 9007199254740992.0
    return u, v


def poisson(lam, p, stream, key, max_tries=64):
    if not lam > 0:
        return 0.0
    if lam < 10:
        u, _ = uniforms2(p, 0, stream, key)
        pk = math.exp(-lam)
        cdf = pk
        k = 0
        while u > cdf and k < 1000:
            k += 1
            pk *= lam / k
            cdf += pk
        return float(k)
    slam, loglam = math.sqrt(lam), math.log(lam)
    b = 0.931 + 2.53 * slam
    a = -0.059 + 0.02483 * b
    invalpha = 1.1239 + 1.1328 / (b - 3.4)
    vr = 0.9277 - 3.6224 / (b - 2.0)
    for t in range(max_tries):
        u, v = uniforms2(p, t, stream, key)
        u -= 0.5
        us = 0.5 - abs(u)
        k = math.floor((2.0 * a / us + b) * u + lam + 0.43)
        if us >= 0.07 and v <= vr:
            return float(k)
        if k < 0 or (us < 0.013 and v > us):
            continue
        if math.log(v) + math.log(invalpha) - math.log(a / (us * us) + b) <= -lam + k * loglam - math.lgamma(k + 1.0):
            return float(k)
    return float(math.floor(lam + 0.5))
