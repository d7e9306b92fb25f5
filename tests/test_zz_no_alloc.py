"""The allocation-free inference entry point against the allocating one,
through the C ABI: bit-identical outputs on two calls in a row (the second
with fewer points, so stale scratch contents would show), the size limit of
the static scratch refused with EINVAL, and n = 0 a no-op."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU, skipped there
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1004_1451_amd import bamg as B  # noqa: E402

MAXN = 1 << 17


def _features(n, seed):
    g = torch.Generator().manual_seed(seed)
    f = torch.randn((n, 24), generator=g, dtype=torch.float32) * 2.0
    f[:, :4] = (torch.rand((n, 4), generator=g) < 0.8).float()      # slot masks
    return f.cuda()


def test_noalloc_forward_matches_forward():
    params = B.mlp_init(7)
    for n, seed in ((MAXN, 1), (1000, 2), (257, 3)):
        print(f"case n={n} seed={seed}", flush=True)
        feat = _features(n, seed)
        want = B.mlp_forward(feat, params)
        out = torch.full((n, 4), float("nan"), dtype=torch.float32, device="cuda")
        B.mlp_forward_noalloc(feat, params, out)
        torch.cuda.synchronize()
        assert torch.equal(out, want), n
    # a second network on the same scratch: the packed weights are rewritten
    p2 = B.mlp_init(11)
    feat = _features(300, 4)
    out = torch.empty((300, 4), dtype=torch.float32, device="cuda")
    B.mlp_forward_noalloc(feat, p2, out)
    assert torch.equal(out, B.mlp_forward(feat, p2))


def test_noalloc_forward_limits():
    lib = B.load()
    params = torch.zeros(B.MLP_NPARAM, dtype=torch.float32, device="cuda")
    out = torch.zeros((1, 4), dtype=torch.float32, device="cuda")
    feat = torch.zeros((1, 24), dtype=torch.float32, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.bamg_mlp_forward_noalloc(C.c_void_p(feat.data_ptr()), MAXN + 1, C.c_void_p(params.data_ptr()),
                                      C.c_void_p(out.data_ptr()), s)
    assert rc == B.EINVAL and b"scratch" in lib.bamg_last_error()
    rc = lib.bamg_mlp_forward_noalloc(None, 1, C.c_void_p(params.data_ptr()), C.c_void_p(out.data_ptr()), s)
    assert rc == B.EINVAL
    assert lib.bamg_mlp_forward_noalloc(C.c_void_p(feat.data_ptr()), 0, C.c_void_p(params.data_ptr()),
                                        C.c_void_p(out.data_ptr()), s) == B.OK
