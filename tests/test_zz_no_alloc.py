"""riga_project_noalloc (the Gram-Schmidt pass with its workspace in the
library's fixed per-GPU scratch array) against riga_project (the same
kernels with an allocated workspace): bitwise equal results on two calls in
a row, the second with a smaller input, so the second reads scratch that
the first left behind; sizes beyond the scratch are refused."""
import ctypes as C
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _riga():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_08167_amd import riga
    riga.lib()
    return riga


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n, m, seed):
    rng = np.random.default_rng(seed)
    W = torch.tensor(rng.standard_normal((m, n)), device="cuda")
    B = torch.tensor(rng.standard_normal((m, n)), device="cuda")
    x = torch.tensor(rng.standard_normal(n), device="cuda")
    return W, B, x


def test_noalloc_equals_allocating_entry_point_twice():
    riga = _riga()
    for n, m, seed in ((82369, 300, 1), (5000, 7, 2)):
        _say("noalloc project", n, m)
        W, B, x = _case(n, m, seed)
        x_ref, x_na = x.clone(), x.clone()
        c_ref = riga.project(W, B, x_ref)
        c_na = riga.project(W, B, x_na, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(c_na, c_ref), (n, m)
        assert torch.equal(x_na, x_ref), (n, m)


def test_noalloc_queued_back_to_back_on_one_stream():
    """Calls on one stream run in order: two passes queued without a host
    synchronisation equal two allocating passes."""
    riga = _riga()
    W, B, x = _case(20000, 64, 3)
    x1, x2 = x.clone(), x.clone()
    riga.project(W, B, x1)
    riga.project(W, B, x1)
    riga.project(W, B, x2, noalloc=True)
    riga.project(W, B, x2, noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2)


def test_noalloc_refuses_sizes_beyond_the_scratch():
    riga = _riga()
    L = riga.lib()
    W = torch.zeros((2, 8), dtype=torch.float64, device="cuda")
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    c = torch.zeros(2, dtype=torch.float64, device="cuda")
    p = [C.c_void_p(t.data_ptr()) for t in (W, W, x, c)]
    # ceil(n / 4096) * m doubles of scratch: 2^20 at most (the arrays are
    # not touched when the size is refused)
    for n, m in ((4096 * 129, 8192), (4096 * 1024 + 1, 1024), (0, 1), (8, 0)):
        assert L.riga_project_noalloc(n, m, *p, None) == riga.RIGA_EINVAL, (n, m)
    code = L.riga_project_noalloc(4096 * 129, 8192, *p, None)
    assert code == riga.RIGA_EINVAL and b"exceeds the fixed scratch" in L.riga_last_error()
