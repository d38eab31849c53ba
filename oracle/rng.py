"""Oracle: counter-based random numbers for the setup's test vectors (test infrastructure).

The setup draws random starting test vectors (paper, DDalphaAMG section: random test
vectors relaxed towards D x = 0).  Both the oracle and the GPU library produce them from
the same published counter generator so that no random stream has to be shared:

* splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
  OOPSLA 2014), first output for state s: z = s + 0x9E3779B97F4A7C15;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9; z = (z ^ (z >> 27)) * 0x94D049BB133111EB;
  return z ^ (z >> 31)   (all arithmetic mod 2^64);
* component value u = (hash >> 11) * 2^-52 - 1 in [-1, 1), exact in binary64;
* key = (level << 56) | (k << 40) | (dof << 1) | part, part 0 = real, 1 = imaginary;
  the hashed state is seed XOR key.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def splitmix64_int(state: int) -> int:
    """First splitmix64 output for a Python integer state (arbitrary-precision reference)."""
    z = (state + GOLDEN) & _MASK
    z = ((z ^ (z >> 30)) * M1) & _MASK
    z = ((z ^ (z >> 27)) * M2) & _MASK
    return z ^ (z >> 31)


def splitmix64_sequence(seed: int, count: int) -> list:
    """The generator's stream: state advances by the golden gamma before each output."""
    out, s = [], seed & _MASK
    for _ in range(count):
        out.append(splitmix64_int(s))
        s = (s + GOLDEN) & _MASK
    return out


def splitmix64_np(state: np.ndarray) -> np.ndarray:
    """Vectorised first output for uint64 states (wrapping uint64 arithmetic)."""
    with np.errstate(over="ignore"):
        z = state.astype(np.uint64) + np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        return z ^ (z >> np.uint64(31))


def test_vectors(seed: int, level: int, nv: int, ndof: int) -> np.ndarray:
    """Complex [nv][ndof] array with independent uniform [-1, 1) real and imaginary parts."""
    k = np.arange(nv, dtype=np.uint64)[:, None]
    dof = np.arange(ndof, dtype=np.uint64)[None, :]
    base = (np.uint64(level) << np.uint64(56)) | (k << np.uint64(40)) | (dof << np.uint64(1))
    out = []
    for part in (0, 1):
        key = base | np.uint64(part)
        h = splitmix64_np(np.uint64(seed) ^ key)
        out.append((h >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0)
    return out[0] + 1j * out[1]
