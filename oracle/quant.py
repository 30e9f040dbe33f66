"""Oracle: the bfloat16 rounding that defines the BF16 precision form (test
infrastructure only).

The BF16 form runs the quantised model: every weight W_ji is replaced by its nearest
bfloat16 value (8 significant bits, ties to even) while a, b and all arithmetic stay at
least FP32; the Jacobian contractions of the SR step (O v, O^dagger u) read tanh(theta)
rounded the same way. This module states that rounding from its definition (significand
scaled to 8 bits, rounded half to even) for float64 / complex128 arrays.

Pinned by tests/test_oracle_quant.py: exact ties and representable values, and agreement
with torch's float32 -> bfloat16 conversion on random inputs.
"""
import numpy as np


def bf16(x):
    """Nearest bfloat16 value of each element (ties to even), as float64 / complex128.
    Finite inputs in the normal range of bfloat16 only."""
    x = np.asarray(x)
    if np.iscomplexobj(x):
        return bf16(x.real) + 1j * bf16(x.imag)
    m, e = np.frexp(x.astype(np.float64))      # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def quantize_weights(params, n_sites, n_hidden):
    """Parameters of the quantised model: W rounded to bfloat16, a and b unchanged."""
    p = np.array(params, dtype=np.complex128 if np.iscomplexobj(params) else np.float64)
    off = n_sites + n_hidden
    p[off:] = bf16(p[off:])
    return p
