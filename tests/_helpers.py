"""Shared test helpers (no scheme arithmetic)."""
import numpy as np


def rel_err_per_component(a: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """max_i |a - ref| / max_i |ref| per column."""
    scale = np.abs(ref).max(0)
    scale = np.where(scale > 0, scale, 1.0)
    return np.abs(a - ref).max(0) / scale
