"""Counter-based stratified sample offsets for the oracle (test infrastructure).

The per-sample offset u in [0, 1) inside each depth bin is a hash of
(seed, ray index, hit rank, sample index).  The hash is the 32-bit PCG output
permutation used as a stateless hash, as published by Jarzynski and Olano,
"Hash Functions for GPU Rendering", JCGT 9(3), 2020:

    state = v * 747796405 + 2891336453            (mod 2^32)
    word  = ((state >> ((state >> 28) + 4)) ^ state) * 277803737
    hash  = (word >> 22) ^ word

u = (pcg(pcg(pcg(pcg(seed) + ray) + rank) + k) >> 8) * 2^-24, so u has 24 bits
and is exactly representable in float32.  The HIP library implements the same
definition on its own; only the integers are shared, never code.
"""
import numpy as np

__all__ = ["pcg_hash", "sample_offsets"]


def pcg_hash(v) -> np.ndarray:
    v = np.asarray(v, dtype=np.uint32)
    with np.errstate(over="ignore"):
        state = v * np.uint32(747796405) + np.uint32(2891336453)
        shift = (state >> np.uint32(28)) + np.uint32(4)
        word = ((state >> shift) ^ state) * np.uint32(277803737)
        return (word >> np.uint32(22)) ^ word


def sample_offsets(seed, ray, rank, k) -> np.ndarray:
    """u for each sample (arrays broadcast); float64 holding a float32 value."""
    with np.errstate(over="ignore"):
        h = pcg_hash(np.uint32(seed & 0xFFFFFFFF))
        h = pcg_hash(h + np.asarray(ray, dtype=np.int64).astype(np.uint32))
        h = pcg_hash(h + np.asarray(rank, dtype=np.int64).astype(np.uint32))
        h = pcg_hash(h + np.asarray(k, dtype=np.int64).astype(np.uint32))
    return (h >> np.uint32(8)).astype(np.float64) * (2.0 ** -24)
