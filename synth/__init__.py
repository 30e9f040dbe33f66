"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only draws random numbers and lays
them out. Parameters follow the paper's initialisation (Listing of Sec. 2.2.5:
``init_random_parameters(seed=1234, sigma=0.01)``), read as independent normal draws of
standard deviation ``sigma`` for the real and the imaginary part of every parameter.
Spin configurations are +/-1 int8 rows, optionally in the zero-magnetisation sector.
"""
import numpy as np


def n_params(n_sites, n_hidden):
    return n_sites + n_hidden + n_sites * n_hidden


def rbm_params(n_sites, n_hidden, is_complex, sigma=0.01, seed=1234, dtype=None):
    """Packed [a (N) | b (M) | W (M x N row-major)] parameters, N(0, sigma^2) entries.
    dtype defaults to complex128 / float64; a lower-precision dtype rounds the draws."""
    rng = np.random.default_rng(seed)
    P = n_params(n_sites, n_hidden)
    if is_complex:
        p = rng.normal(0.0, sigma, P) + 1j * rng.normal(0.0, sigma, P)
        return p.astype(dtype or np.complex128)
    return rng.normal(0.0, sigma, P).astype(dtype or np.float64)


def spin_configs(n, n_sites, seed, zero_magnetisation=False):
    """n random configurations [n, N] of +/-1 spins (int8)."""
    rng = np.random.default_rng(seed)
    if not zero_magnetisation:
        return (1 - 2 * rng.integers(0, 2, size=(n, n_sites))).astype(np.int8)
    base = np.array([1] * (n_sites // 2) + [-1] * (n_sites - n_sites // 2), dtype=np.int8)
    out = np.empty((n, n_sites), dtype=np.int8)
    for k in range(n):
        out[k] = rng.permutation(base)
    return out


def random_vector(n, is_complex, seed, dtype=None):
    rng = np.random.default_rng(seed)
    if is_complex:
        return (rng.normal(size=n) + 1j * rng.normal(size=n)).astype(dtype or np.complex128)
    return rng.normal(size=n).astype(dtype or np.float64)


def tfim_instances(n_instances, seed, n_min=16, n_max=128, h_min=0.5, h_max=1.5, even=True):
    """Uneven batch of TFIM rings: sizes uniform in [n_min, n_max] (even when ``even``),
    fields uniform in [h_min, h_max]."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_min, n_max + 1, size=n_instances)
    if even:
        ns = ns - (ns % 2)
        ns = np.maximum(ns, n_min + (n_min % 2))
    hs = rng.uniform(h_min, h_max, size=n_instances)
    return [int(x) for x in ns], [float(x) for x in hs]
