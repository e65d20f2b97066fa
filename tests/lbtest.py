"""Helpers shared by the GPU tests: input quantisation to a storage format and
the error metrics used to compare the GPU path with the FP64 oracle."""

import numpy as np

# power-of-two factors applied to f_i - w_i before 16-bit rounding (interface
# convention of the storage format; defined per direction class)
SCALES = {
    15: np.array([4.0] + [8.0] * 6 + [64.0] * 8),
    19: np.array([4.0] + [16.0] * 6 + [32.0] * 12),
}


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def quantize(delta, q, storage, scale=True):
    """Deviations exactly representable in a storage format (float64 array)."""
    if storage == "f32":
        return delta.astype(np.float32).astype(np.float64)
    s = SCALES[q][:, None] if scale else np.ones((q, 1))
    if storage == "f16":
        return (delta * s).astype(np.float16).astype(np.float64) / s
    if storage == "bf16":
        return bf16_round((delta * s).astype(np.float32)).astype(np.float64) / s
    raise ValueError(storage)


def rel_max(gpu, ref):
    """max |gpu - ref| / max |ref| over sites (vectors use the Euclidean norm)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if gpu.ndim == 2:
        num = np.sqrt(((gpu - ref) ** 2).sum(axis=1)).max()
        den = np.sqrt((ref ** 2).sum(axis=1)).max()
    else:
        num = np.abs(gpu - ref).max()
        den = np.abs(ref).max()
    return num / den if den > 0 else num


def rel_l2(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return np.linalg.norm(gpu - ref) / den if den > 0 else np.linalg.norm(gpu - ref)
