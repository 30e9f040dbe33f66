"""Pins of the oracle's bfloat16 rounding (CPU)."""
import numpy as np
import torch

from oracle import quant


def test_exact_cases():
    # spacing of bfloat16 at 1 is 2^-7
    assert quant.bf16(1.0) == 1.0
    assert quant.bf16(1.0 + 2.0 ** -8) == 1.0                     # tie -> even (1.0)
    assert quant.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie -> even (mantissa 2)
    assert quant.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert quant.bf16(-3.0) == -3.0
    assert quant.bf16(0.0) == 0.0
    assert quant.bf16(2.0 ** -100) == 2.0 ** -100
    z = quant.bf16(np.array([1.0 + 2.0 ** -8 + 1j * (1.0 + 3 * 2.0 ** -8)]))
    assert z[0] == 1.0 + 1j * (1.0 + 2.0 ** -6)


def test_matches_library_conversion():
    rng = np.random.default_rng(0)
    x = (rng.normal(size=20000) * np.exp(rng.uniform(-20, 20, size=20000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(quant.bf16(x.astype(np.float64)), ref)


def test_quantize_weights_only_touches_w():
    rng = np.random.default_rng(1)
    N, M = 5, 7
    p = rng.normal(size=N + M + N * M) + 1j * rng.normal(size=N + M + N * M)
    q = quant.quantize_weights(p, N, M)
    assert np.array_equal(q[:N + M], p[:N + M])
    assert np.array_equal(q[N + M:], quant.bf16(p[N + M:]))
    assert np.abs(q[N + M:] - p[N + M:]).max() <= 2.0 ** -8 * np.abs(p[N + M:]).max() * 1.5
