"""Counter-based random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).

Value i of stream s under seed k is the SplitMix64 output for the state
key(k, s) + (i + 1) * gamma, where gamma = 0x9E3779B97F4A7C15 and
key(k, s) = mix64(k + (s + 1) * gamma).  Every array is therefore a pure
function of (seed, stream, index) and can be regenerated piecewise.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Named streams, so that geometry, noise and right-hand sides never share draws.
STREAMS = {"geom": 1, "jitter": 2, "rhs": 3, "dirs": 4, "noise": 5, "target": 6, "sizes": 7,
           "entries": 8, "hubs": 9}


def mix64(z):
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _stream_id(stream):
    return STREAMS[stream] if isinstance(stream, str) else int(stream)


def raw64(seed, stream, count, offset=0):
    """uint64 draws [offset, offset+count) of one stream."""
    with np.errstate(over="ignore"):
        key = mix64(np.array([np.uint64(seed) + np.uint64(_stream_id(stream) + 1) * _GAMMA],
                             dtype=np.uint64))[0]
        idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        return mix64(key + idx * _GAMMA)


def uniform(seed, stream, count, lo=0.0, hi=1.0, offset=0):
    """53-bit uniforms on [lo, hi)."""
    u = (raw64(seed, stream, count, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return lo + (hi - lo) * u


def normal(seed, stream, count, offset=0):
    """Standard normals by Box-Muller from two consecutive uniforms per value."""
    u = uniform(seed, stream, 2 * count, offset=2 * offset)
    u1 = 1.0 - u[0::2]          # (0, 1]: keeps log finite
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
