"""Counter-based noise for the inlet fluctuations, from the published SplitMix64 mixing
function (Steele, Lea, Flood, OOPSLA 2014), in numpy uint64 (wrapping) arithmetic.

xi(seed, a, b, n) is uniform on [-sqrt(3), sqrt(3)) (zero mean, unit variance) for the
inlet-face cell with in-face coordinates (a, b) at step n:
  ctr = (n << 40) | (b << 20) | a
  z = seed + ctr * 0x9E3779B97F4A7C15
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
  z = (z ^ (z >> 27)) * 0x94D049BB133111EB
  z = z ^ (z >> 31)
  U = (z >> 11) * 2^-53 ;  xi = sqrt(3) (2U - 1)
"""
import numpy as np


def xi(seed, a, b, n):
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = (np.uint64(n) << np.uint64(40)) | (b << np.uint64(20)) | a
        z = np.uint64(seed) + ctr * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    U = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return np.sqrt(3.0) * (2.0 * U - 1.0)


def raw(seed, ctr):
    """The 64-bit SplitMix64 output for counter value ctr (Python integers)."""
    m = 0xFFFFFFFFFFFFFFFF
    z = (seed + ctr * 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)
