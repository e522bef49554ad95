"""The no-allocation FP32 solve (sr_trisolve_static) against sr_trisolve, through
the C interface: the same kernels, so the same L bit for bit and the same
breakdown outcome, on two calls in a row (the second smaller, so that it runs on
what the first left in the library's fixed scratch array)."""
import numpy as np
import pytest

import synth
from gpu_util import dev, empty, host, rand_c

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sr():
    import torch

    import paper_2203_10879_amd as m

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _case(n, seed):
    rng = np.random.default_rng(seed)
    g = synth.schur_test_matrix(n, seed=seed)
    t = np.asfortranarray(np.triu(g["T0"]).astype(np.complex64))
    e = np.asfortranarray((1e-6 * np.tril(rand_c(rng, (n, n)), -1)).astype(np.complex64))
    return t, e


def _flag():
    import torch

    return torch.full((1,), 12345, dtype=torch.int32, device="cuda")


@pytest.mark.parametrize("sizes", [(2100, 300), (1024, 33)])
def test_static_solve_matches_workspace_solve(sr, sizes):
    import torch

    for n in sizes:
        t, e = _case(n, 500 + n)
        td, ed = dev(t), dev(e)
        ref = empty(n, n, True)
        assert sr.sr_trisolve(td, ed, ref, sr.workspace(n)) == 0
        out = empty(n, n, True)
        flag = _flag()
        assert sr.sr_trisolve_static(td, ed, out, flag) == 0
        torch.cuda.synchronize()
        assert int(flag.item()) == 0
        assert np.array_equal(host(out), host(ref)), n


def test_static_solve_truncation_and_breakdown(sr):
    import torch

    t, e = _case(70, 9)
    e = np.asfortranarray(e * np.complex64(1e6))
    ref = empty(70, 70, True)
    assert sr.sr_trisolve(dev(t), dev(e), ref, sr.workspace(70), trunc=1e-5) == 0
    out, flag = empty(70, 70, True), _flag()
    assert sr.sr_trisolve_static(dev(t), dev(e), out, flag, trunc=1e-5) == 0
    torch.cuda.synchronize()
    assert int(flag.item()) == 0 and np.array_equal(host(out), host(ref))
    # Theorem 1: two equal diagonal entries make the equation singular
    t = np.triu(np.ones((40, 40), dtype=np.complex64))
    t[np.diag_indices(40)] = np.arange(40)
    t[35, 35] = t[3, 3]
    e = np.asfortranarray(np.tril(np.ones((40, 40), dtype=np.complex64), -1))
    t = np.asfortranarray(t)
    assert sr.sr_trisolve(dev(t), dev(e), empty(40, 40, True), sr.workspace(40)) == 3
    flag = _flag()
    assert sr.sr_trisolve_static(dev(t), dev(e), empty(40, 40, True), flag) == 0
    torch.cuda.synchronize()
    assert int(flag.item()) != 0


def test_static_solve_rejects_sizes_beyond_its_array(sr):
    import torch

    n = 4097
    t = torch.zeros((n, 1), dtype=torch.complex64, device="cuda")
    # validation happens before any pointer is used, so 1-column stand-ins suffice
    lib = sr.lib()
    import ctypes

    flag = _flag()
    p = ctypes.c_void_p(t.data_ptr())
    assert lib.sr_trisolve_static(p, p, p, n, 0.0, ctypes.c_void_p(flag.data_ptr()), None) == -3
    assert lib.sr_trisolve_static(p, p, p, 0, 0.0, ctypes.c_void_p(flag.data_ptr()), None) == -1
    assert lib.sr_trisolve_static(p, p, p, 16, 0.0, None, None) == -1
    torch.cuda.synchronize()
    assert int(flag.item()) == 12345  # nothing ran
