"""Small test-side helpers: input rounding, error norms, and the choice of oracle reference for a
rounded GPU path (no decomposition arithmetic of their own)."""
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


def bf16_matrix_core_path(dims, ranks, mode) -> bool:
    """Whether a BF16 TTMc of this mode runs on the BF16 matrix instruction: order 3 with both
    other ranks at most 16 (the library's rule for its order-3 kernel)."""
    return len(dims) == 3 and all(r <= 16 for t, r in enumerate(ranks) if t != mode)


def oracle_ttmc_rounded(coords, vals, dims, ranks, mode, U, dtype):
    """The oracle's TTMc on the inputs as the GPU path holds them (values and factors rounded to
    the storage type); on the BF16 matrix-core path also with each product x a rounded to BF16,
    the one rounding that path adds.  What remains against the GPU is FP32 accumulation order."""
    import oracle
    v, Uc = cast_vals(vals, dtype), cast_inputs(U, dtype)
    if dtype == "bf16" and bf16_matrix_core_path(dims, ranks, mode):
        return oracle.ttmc_bf16_operands(coords, v, dims, ranks, mode, Uc)
    return oracle.ttmc(coords, v, dims, ranks, mode, Uc)

