"""nqs_log_psi_grad_noalloc (scratch in the library's fixed per-device array, no
allocation) against nqs_log_psi_grad: two calls in a row, the second with fewer samples,
bit for bit; sizes beyond the array are rejected before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import cases

pytestmark = pytest.mark.gpu

DEV = "cuda"


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("name", ["heis40_cplx_f32", "tfim10_real_f64", "j1j2_4x4_cplx_bf16"])
def test_noalloc_matches_log_psi_grad(lib, name):
    m, om = cases.build(lib, name)
    p = to_dev(cases.params(name, seed=501))
    rng = np.random.default_rng(502)
    for n in (5000, 1203):
        s = to_dev(cases.configs(name, n, seed=503 + n))
        P = m.n_params
        if m.is_complex:
            u = to_dev(rng.normal(size=n) + 1j * rng.normal(size=n))
            v = to_dev(rng.normal(size=P) + 1j * rng.normal(size=P))
        else:
            u = to_dev(rng.normal(size=n))
            v = to_dev(rng.normal(size=P))
        vjp_a, jvp_a = m.log_psi_grad(p, s, u=u, v=v)
        vjp_b = torch.full_like(vjp_a, float("nan"))
        jvp_b = torch.full_like(jvp_a, float("nan"))
        m.log_psi_grad(p, s, u=u, v=v, vjp=vjp_b, jvp=jvp_b, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(vjp_a, vjp_b), (name, n)
        assert torch.equal(jvp_a, jvp_b), (name, n)


def test_noalloc_rejects_sizes_beyond_its_scratch(lib):
    m, om = cases.build(lib, "heis40_cplx_f32")
    p = to_dev(cases.params("heis40_cplx_f32", seed=504))
    n = 400000   # 400,000 x 80 complex FP32 rows alone exceed 64 MiB
    s = torch.ones((n, 40), dtype=torch.int8, device=DEV)
    u = torch.zeros(n, dtype=torch.complex128, device=DEV)
    out = torch.zeros(m.n_params, dtype=torch.complex128, device=DEV)
    st = lib._lib.nqs_log_psi_grad_noalloc(m._h, ctypes.c_void_p(p.data_ptr()),
                                           ctypes.c_void_p(s.data_ptr()), n,
                                           ctypes.c_void_p(u.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), None, None,
                                           lib._stream())
    assert st == lib.ENOMEM
    assert lib._lib.nqs_log_psi_grad_noalloc(None, None, None, 4, None, None, None, None,
                                             None) == lib.EINVAL
