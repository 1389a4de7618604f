"""Round-to-nearest-even onto the bfloat16 and float32 value grids (test infrastructure).

Written from the formats' definitions: a binary floating-point format with p significand bits
(implicit bit included) and exponent range [emin, emax] represents, in the binade
[2^e, 2^(e+1)) with emin <= e <= emax, exactly the multiples of 2^(e - p + 1); below 2^emin
(subnormals) the multiples of 2^(emin - p + 1).  Rounding picks the nearest grid value, ties to
the one with an even multiple, and magnitudes that round beyond the largest finite value become
infinity.  bfloat16 is p = 8, float32 is p = 24, both with emin = -126, emax = 127.

The GPU path stores BF16 tensors; the oracle's emulating mode applies these roundings exactly
where the GPU stores a value, to separate kernel bugs from quantisation.
"""
import numpy as np


def _round_to_grid(x, p: int, emin: int, emax: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    out = np.array(x, copy=True)
    finite = np.isfinite(x) & (x != 0.0)
    xf = x[finite]
    _, e2 = np.frexp(xf)                  # |x| in [2^(e2-1), 2^e2)
    e = np.maximum(e2 - 1, emin)          # binade exponent, clamped at the subnormal range
    spacing = np.ldexp(1.0, e - p + 1)
    y = np.round(xf / spacing) * spacing  # np.round: half to even; scaling by 2^k is exact
    max_finite = (2.0 - 2.0 ** (1 - p)) * 2.0 ** emax
    y = np.where(np.abs(y) > max_finite, np.copysign(np.inf, y), y)
    out[finite] = y
    return out


def round_bf16(x) -> np.ndarray:
    """Nearest bfloat16 value (ties to even) of each element, returned as float64."""
    return _round_to_grid(x, 8, -126, 127)


def round_f32(x) -> np.ndarray:
    """Nearest float32 value (ties to even) of each element, returned as float64."""
    return _round_to_grid(x, 24, -126, 127)


def round_to(x, dtype: str) -> np.ndarray:
    """Round to the storage dtype named in a DAG spec ("f32" or "bf16")."""
    if dtype == "bf16":
        return round_bf16(x)
    if dtype == "f32":
        return round_f32(x)
    raise ValueError(f"unknown dtype {dtype!r}")
