"""Storage rounding of matrix blocks (a project addition: the paper states no precision).

Blocks are rounded from FP64 to the storage format with round-to-nearest, ties to even,
directly from the double value (no intermediate format):
  FP32: 24 significant bits (numpy's float64 -> float32 cast is exactly this rounding);
  BF16: 8 significant bits, FP32 exponent range.  Implemented with frexp: for
        x = m 2^e with 0.5 <= |m| < 1, the BF16 value is rint(m 2^8) 2^(e-8)
        (numpy's rint rounds half to even).  Magnitudes below 2^-126 (BF16 subnormals)
        and above the BF16 range do not occur in the matrices here; they raise.
The "stored" operator of the reduced-precision modes is the FP64 upcast of these values.
"""
import numpy as np


def round_fp32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    x = np.asarray(x, np.float64)
    nz = x != 0
    ax = np.abs(x[nz])
    if ax.size and (ax.min() < 2.0 ** -126 or ax.max() >= 3.3e38):
        raise ValueError("value outside the normal BF16 range")
    m, e = np.frexp(x)
    return np.rint(m * 256.0) * np.exp2(e.astype(np.float64) - 8.0)


def round_storage(x, storage):
    if storage in ("f64", "FP64"):
        return np.asarray(x, np.float64).copy()
    if storage in ("f32", "FP32"):
        return round_fp32(x)
    if storage in ("bf16", "BF16"):
        return round_bf16(x)
    raise ValueError(storage)
