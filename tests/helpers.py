"""Small test-side helpers (no decomposition arithmetic)."""
import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """float64 -> float32 -> bf16 bits with round-to-nearest-even (as int16 bit patterns)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return r.view(np.int16)


def bf16_value(x: np.ndarray) -> np.ndarray:
    """float64 -> nearest bf16 value, returned as float64."""
    b = bf16_round(x).view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def rel_fro(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def cast_inputs(U, dtype):
    """Factors as the GPU path's TTMc sees them (FP64 values rounded to the TTMc storage type)."""
    if dtype == "f64":
        return [np.asarray(u, dtype=np.float64) for u in U]
    if dtype == "f32":
        return [np.asarray(u, dtype=np.float32).astype(np.float64) for u in U]
    return [bf16_value(u) for u in U]


def cast_vals(v, dtype):
    if dtype == "f64":
        return np.asarray(v, dtype=np.float64)
    if dtype == "f32":
        return np.asarray(v, dtype=np.float32).astype(np.float64)
    return bf16_value(v)
