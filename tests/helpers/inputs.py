"""Seeded synthetic inputs shared by oracle and GPU tests (no lattice
arithmetic here): link-angle arrays uniform in [-pi, pi)."""
import numpy as np


def random_links(volume: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, 4 * volume)


def random_links_fp32(volume: int, seed: int) -> np.ndarray:
    """Angles exactly representable in FP32 (for FP32-storage comparisons)."""
    return random_links(volume, seed).astype(np.float32).astype(np.float64)
