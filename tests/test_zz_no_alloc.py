"""The allocation-free network gradient (acopf_mlp_gradient_noalloc) against
the gradient with a caller-supplied scratch buffer (acopf_mlp_gradient),
through the C ABI: same kernels and reduction order, so the same bits; two
calls in a row, the second with fewer samples and a smaller network, so a
stale partial from the first call would show."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(lib, torch, n_in, n_out, n, seed):
    from paper_2310_13143_amd._abi import check
    from paper_2310_13143_amd.warmstart import init_params
    print(f"[gpu] noalloc gradient n_in={n_in} n_out={n_out} n={n}", flush=True)
    rng = np.random.default_rng(seed)
    count = int(lib.acopf_mlp_param_count(n_in, n_out))
    theta = torch.as_tensor(init_params(n_in, n_out, seed) + rng.normal(0, 0.05, count).astype(np.float32)).cuda()
    ld = n + 5
    X = torch.as_tensor(rng.standard_normal((n_in, ld)).astype(np.float32)).cuda()
    T = torch.as_tensor(rng.standard_normal((n_out, ld)).astype(np.float32)).cuda()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    need = int(lib.acopf_mlp_scratch_bytes(n_in, n_out, n))
    scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
    g_ref = torch.empty(count, dtype=torch.float32, device="cuda")
    l_ref = torch.empty(1, dtype=torch.float32, device="cuda")
    check(lib.acopf_mlp_gradient(theta.data_ptr(), n_in, n_out, X.data_ptr(), ld, T.data_ptr(), ld, n,
                                 g_ref.data_ptr(), l_ref.data_ptr(), scratch.data_ptr(), need, stream))
    g = torch.full((count,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    check(lib.acopf_mlp_gradient_noalloc(theta.data_ptr(), n_in, n_out, X.data_ptr(), ld, T.data_ptr(), ld, n,
                                         g.data_ptr(), loss.data_ptr(), stream))
    torch.cuda.synchronize()
    a, b = g.cpu().numpy(), g_ref.cpu().numpy()
    assert np.isfinite(a).all() and np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert loss.item() == l_ref.item() and np.isfinite(loss.item())


def test_noalloc_gradient_equals_the_scratch_gradient():
    import torch
    from paper_2310_13143_amd import _abi
    lib = _abi.load()
    # the most blocks and the largest network first, then a small call
    _case(lib, torch, 64, 16, 40000, 1)
    _case(lib, torch, 7, 3, 150, 2)


def test_noalloc_rejects_bad_sizes():
    import torch
    from paper_2310_13143_amd import _abi
    lib = _abi.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    x = torch.zeros(16, device="cuda")
    rc = lib.acopf_mlp_gradient_noalloc(x.data_ptr(), 65, 4, x.data_ptr(), 4, x.data_ptr(), 4, 4, x.data_ptr(),
                                        x.data_ptr(), stream)
    assert rc == -1  # ACOPF_ERR_INVALID_ARG
    rc = lib.acopf_mlp_gradient_noalloc(x.data_ptr(), 4, 4, x.data_ptr(), 2, x.data_ptr(), 4, 4, x.data_ptr(),
                                        x.data_ptr(), stream)
    assert rc == -1  # ACOPF_ERR_INVALID_ARG
