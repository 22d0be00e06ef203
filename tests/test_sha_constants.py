"""The SHA-256 constants of the device fingerprint kernel against their definition in FIPS 180-4: K[i] is the first
32 bits of the fractional part of the cube root of the i-th prime (Sec. 4.2.2), H0[i] of the square root of the i-th
prime (Sec. 5.3.3).  Computed here with exact integer roots, so a mistyped constant fails without a GPU."""
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "paper_2505_21194_amd", "csrc", "seqcdc_fingerprint.hip")


def _primes(k):
    out, n = [], 2
    while len(out) < k:
        if all(n % p for p in out if p * p <= n):
            out.append(n)
        n += 1
    return out


def _iroot(x, k):
    """floor(x ** (1/k)) for a non-negative integer x, exactly."""
    r = int(round(x ** (1.0 / k)))
    while r ** k > x:
        r -= 1
    while (r + 1) ** k <= x:
        r += 1
    return r


def _table(name):
    src = open(SRC).read()
    m = re.search(name + r"\[\d+\]\s*=\s*\{(.*?)\};", src, re.S)
    assert m, name
    return [int(v, 16) for v in re.findall(r"0x([0-9a-fA-F]+)u", m.group(1))]


def test_round_constants():
    want = [_iroot(p << 96, 3) & 0xFFFFFFFF for p in _primes(64)]  # floor(cbrt(p) * 2^32) mod 2^32
    assert _table("kSha256K") == want


def test_initial_hash_value():
    want = [_iroot(p << 64, 2) & 0xFFFFFFFF for p in _primes(8)]  # floor(sqrt(p) * 2^32) mod 2^32
    assert _table("kSha256H0") == want
