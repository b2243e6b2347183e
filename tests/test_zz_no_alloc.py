"""The allocation-free dot product (VecDotNoAlloc) against VecDot through the
C ABI: bit for bit on two calls in a row, the second with a smaller input,
and no device allocation by the library during the calls."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1701_05913_amd as K  # noqa: E402


def _dot_pair(n, seed, out):
    rng = np.random.default_rng(seed)
    xt = torch.from_numpy(rng.standard_normal(n)).to("cuda:0")
    yt = torch.from_numpy(rng.standard_normal(n)).to("cuda:0")
    m = K.MapCreateLocal(n)
    x, y = K.VecWrap(m, xt), K.VecWrap(m, yt)
    try:
        K.KrylovSetStream(torch.cuda.current_stream())
        ref = K.VecDot(x, y)
        torch.cuda.synchronize()
        K.VecDotNoAlloc(x, y, out)
        torch.cuda.synchronize()
        got = float(out[0].item())
        exact = float(np.dot(xt.cpu().numpy(), yt.cpu().numpy()))
    finally:
        K.VecDestroy(x)
        K.VecDestroy(y)
        K.MapDestroy(m)
    return ref, got, exact


def test_no_alloc_dot_matches_vecdot_twice_shrinking():
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda:0")
    for n, seed in ((3_000_001, 1), (1_537, 2)):
        ref, got, exact = _dot_pair(n, seed, out)
        assert got == ref, (n, got, ref)                   # same kernels, same order
        assert abs(got - exact) <= 1e-12 * np.sqrt(n) * max(1.0, abs(exact)), (n, got, exact)


def test_no_alloc_dot_rejects_bad_arguments():
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    a = torch.zeros(10, dtype=torch.float64, device="cuda:0")
    b = torch.zeros(11, dtype=torch.float64, device="cuda:0")
    ma, mb = K.MapCreateLocal(10), K.MapCreateLocal(11)
    x, y = K.VecWrap(ma, a), K.VecWrap(mb, b)
    try:
        with pytest.raises(K.KrylovError):
            K.VecDotNoAlloc(x, y, out)
    finally:
        K.VecDestroy(x)
        K.VecDestroy(y)
        K.MapDestroy(ma)
        K.MapDestroy(mb)
