"""Counter-based random numbers from the splitmix64 finalizer.

splitmix64 is the generator of Steele, Lea and Flood ("Fast splittable
pseudorandom number generators", OOPSLA 2014).  Its output function takes a
64-bit state z and returns

    z ^= z >> 30;  z *= 0xbf58476d1ce4e5b9
    z ^= z >> 27;  z *= 0x94d049bb133111eb
    z ^= z >> 31

Used here in counter mode: the value for (seed, stream, index) is the output
function applied to seed + GAMMA * (stream * 2**32 + index + 1), all mod 2**64,
where GAMMA = 0x9e3779b97f4a7c15 is the generator's golden-ratio increment.
Every random quantity of a workload draws from its own stream, so any element
can be regenerated on its own.
"""

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB

#: base seed of every workload (the arXiv number of the thesis)
BASE_SEED = 190805845


def splitmix64_mix(z):
    """Output function of splitmix64 on uint64 numpy arrays (wrapping)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z ^ (z >> np.uint64(30))
        z = z * np.uint64(M1)
        z = z ^ (z >> np.uint64(27))
        z = z * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return z


def _mix_int(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def config_seed(c: int) -> int:
    """Seed of workload number c: the output function applied to BASE_SEED + c."""
    return _mix_int(BASE_SEED + c)


def raw(seed: int, stream: int, idx) -> np.ndarray:
    """uint64 draws for the given indices of one stream."""
    idx = np.asarray(idx, dtype=np.uint64)
    ctr = (np.uint64((stream << 32) & MASK64) + idx + np.uint64(1))
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + np.uint64(GAMMA) * ctr
    return splitmix64_mix(z)


def uniform(seed: int, stream: int, idx) -> np.ndarray:
    """Uniform doubles in [0, 1): the top 53 bits of each draw times 2**-53."""
    return (raw(seed, stream, idx) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, stream: int, idx) -> np.ndarray:
    """Standard normal doubles by the Box-Muller transform of streams 2s and 2s+1."""
    u1 = uniform(seed, 2 * stream, idx)
    u2 = uniform(seed, 2 * stream + 1, idx)
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
