"""The allocation-free gradient entry point (pb_mlp_grad_noalloc, for callers
that cannot allocate device memory) against pb_mlp_grad, called through the
C ABI: two calls in a row, the second on a smaller batch (the shared scratch
keeps the first call's partial rows, which the second must not read)."""
import ctypes as C

import numpy as np
import pytest

from oracle import mlp as M
import paper_2608_19273_amd as pb
from paper_2608_19273_amd import inputs as I

from gpu_helpers import announce, need_gpu

pytestmark = pytest.mark.gpu


def test_grad_noalloc_matches_grad():
    torch = need_gpu()
    L = pb.lib()
    vp = C.c_void_p
    L.pb_mlp_grad_noalloc.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp]
    L.pb_mlp_grad_noalloc.restype = C.c_int
    p = (I.normal(81, M.NPARAM) * 0.3).astype(np.float32)
    norm = np.array([-1.0, 0.4, -0.8, -1.5, 0.3, 1.2, 0.3, 0.9, 1.1, 0.25, -3.0, 2.5], np.float32)
    net = pb.Mlp(p, norm)
    for n in (40000, 777):
        announce(f"grad noalloc n={n}")
        x = torch.from_numpy((I.normal(82 + n, n * 5).reshape(n, 5) * 0.8 + norm[:5]).astype(np.float32)).cuda()
        t = torch.from_numpy(I.normal(83 + n, n).astype(np.float32)).cuda()
        g_ref, l_ref = net.grad(x, t)
        g = torch.full((M.NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        rc = L.pb_mlp_grad_noalloc(net.handle, vp(x.data_ptr()), vp(t.data_ptr()), n, vp(g.data_ptr()),
                                   vp(loss.data_ptr()), vp(torch.cuda.current_stream().cuda_stream))
        assert rc == 0, pb.last_error()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(g.cpu().numpy(), g_ref.cpu().numpy())
        np.testing.assert_array_equal(loss.cpu().numpy(), l_ref.cpu().numpy())
    # beyond the stated maximum: rejected before any launch
    rc = L.pb_mlp_grad_noalloc(net.handle, vp(x.data_ptr()), vp(t.data_ptr()), (1 << 30) + 1, vp(g.data_ptr()),
                               vp(loss.data_ptr()), None)
    assert rc == pb.PB_EINVAL and "maximum" in pb.last_error()
    net.close()
