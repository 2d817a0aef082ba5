"""Counter-based SplitMix64 streams (Steele, Lea & Flood, OOPSLA 2014).

Value ``i`` of stream ``sid`` under ``seed`` is the SplitMix64 output function
applied to ``s + (i + 1) * gamma`` with ``s = seed ^ (sid << 48)`` and
``gamma = 0x9E3779B97F4A7C15`` (the golden-ratio increment of the published
generator).  Uniform doubles use the top 53 bits.  Being counter based, any
element of any stream can be produced independently, in any language, from
this definition alone.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_bits(seed, sid, count, start=0):
    """Raw 64-bit outputs ``start .. start+count-1`` of stream ``sid``."""
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ (np.uint64(sid & 0xFFFF) << np.uint64(48))
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(s + i * _GAMMA)


def splitmix64_uniform(seed, sid, count, start=0):
    """Uniform doubles in [0, 1): ``(bits >> 11) * 2**-53``."""
    b = splitmix64_bits(seed, sid, count, start)
    return (b >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform(seed, sid, count, lo=0.0, hi=1.0):
    return lo + (hi - lo) * splitmix64_uniform(seed, sid, count)


def normal(seed, sid, count):
    """Standard normals by Box-Muller on consecutive uniform pairs (u0, u1):
    z0 = sqrt(-2 ln(1-u0)) cos(2 pi u1), z1 = sqrt(-2 ln(1-u0)) sin(2 pi u1)."""
    npair = (count + 1) // 2
    u = splitmix64_uniform(seed, sid, 2 * npair)
    u0, u1 = u[0::2], u[1::2]
    rad = np.sqrt(-2.0 * np.log1p(-u0))
    z = np.empty(2 * npair)
    z[0::2] = rad * np.cos(2.0 * np.pi * u1)
    z[1::2] = rad * np.sin(2.0 * np.pi * u1)
    return z[:count]
