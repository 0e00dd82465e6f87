"""The allocation-free misfit entry point (sbp_nn_mse_noalloc, static device
scratch) against the workspace version (sbp_nn_mse), called through the C
ABI: two calls in a row, the second smaller, and the rejection of a size
beyond its scratch."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(n, y, t, dy, scale):
    from paper_2011_02600_amd import nn
    loss = ctypes.c_double(0)
    rc = nn.lib().sbp_nn_mse_noalloc(n, y.data_ptr(), t.data_ptr(), None if dy is None else dy.data_ptr(), scale,
                                     ctypes.byref(loss), torch.cuda.current_stream().cuda_stream)
    return rc, loss.value


def _workspace(n, y, t, dy, scale):
    from paper_2011_02600_amd import nn
    part = torch.zeros(256, dtype=torch.float64, device="cuda")
    loss = ctypes.c_double(0)
    rc = nn.lib().sbp_nn_mse(n, y.data_ptr(), t.data_ptr(), None if dy is None else dy.data_ptr(), scale,
                             part.data_ptr(), ctypes.byref(loss), torch.cuda.current_stream().cuda_stream)
    return rc, loss.value


def test_mse_noalloc_equals_workspace_version():
    from paper_2011_02600_amd import nn
    g = torch.Generator(device="cpu").manual_seed(5)
    for n in (3_000_017, 1000):  # the second call is smaller and reuses the scratch
        say("case: sbp_nn_mse_noalloc n = %d" % n)
        y = torch.randn(n, generator=g).cuda()
        t = torch.randn(n, generator=g).cuda()
        dy_a = torch.full((n,), float("nan"), device="cuda")
        dy_b = torch.full((n,), float("nan"), device="cuda")
        rc_a, la = _noalloc(n, y, t, dy_a, 0.37)
        rc_b, lb = _workspace(n, y, t, dy_b, 0.37)
        assert rc_a == 0, nn.lib().sbp_nn_last_error().decode()
        assert rc_b == 0
        # the kernels round y - t to float32 and square and sum in double
        want = 0.5 * float(((y - t).double() ** 2).sum())
        say("  loss no-alloc %.17g workspace %.17g float64 %.17g" % (la, lb, want))
        assert abs(la - lb) <= 1e-12 * abs(lb)
        assert abs(la - want) <= 1e-9 * abs(want)
        assert torch.equal(dy_a, dy_b)
        rc_c, lc = _noalloc(n, y, t, None, 1.0)
        assert rc_c == 0 and lc == la
    # one element past the scratch's capacity: rejected on the host, nothing launched
    small = torch.zeros(4, device="cuda")
    big = 65536 * 1024 + 1
    rc, _ = _noalloc(big, small, small, None, 1.0)
    msg = nn.lib().sbp_nn_last_error().decode()
    say("  n = %d: code %d, %s" % (big, rc, msg))
    assert rc == -1 and "67108864" in msg
