"""Counter-based uniform numbers from the SplitMix64 generator.

The eigenvalue estimate of every multigrid level starts from a random vector
(Sec. 4.1: 15 conjugate gradient iterations estimate the largest eigenvalue).
Both the oracle and the GPU library draw it from SplitMix64 (Steele, Lea and
Flood, OOPSLA 2014), each from its own implementation of the published
definition: value i of stream `key` is

    z = key + (i + 1) * 0x9E3779B97F4A7C15  (mod 2^64)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

mapped to [-1, 1) as 2 * (z >> 11) * 2^-53 - 1.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(key, count):
    with np.errstate(over="ignore"):
        i = np.arange(1, int(count) + 1, dtype=np.uint64)
        z = np.uint64(key) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform_pm1(key, count):
    z = splitmix64(key, count)
    return 2.0 * (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 - 1.0
