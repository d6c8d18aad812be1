"""cnmf_spa_noalloc (the entry point that allocates nothing) against cnmf_spa
through the C ABI: the same indices and scores, on two calls in a row (the
second smaller, so stale scratch contents from the first must not leak into
it), for FP64 and FP32 B, and a clear error beyond the fixed scratch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1505_04650_amd import _lib as L  # noqa: E402
from paper_1505_04650_amd import api  # noqa: E402

DEV = torch.device("cuda", 0)


def _b(k, n, seed, dtype):
    g = np.random.default_rng(seed)
    return torch.as_tensor(g.standard_normal((k, n)), dtype=dtype, device=DEV)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_spa_equals_spa_on_two_calls(dtype):
    h = api.Handle(0)
    try:
        for (k, n, r, seed) in ((30, 100000, 20, 1), (12, 5001, 9, 2)):
            B = _b(k, n, seed, dtype)
            K1, s1 = api.spa(B, r, want_scores=True, handle=h)
            K2 = torch.full((r,), -1, dtype=torch.int64, device=DEV)
            s2 = torch.full((r,), -1.0, dtype=torch.float64, device=DEV)
            api.spa(B, r, noalloc=True, K=K2, score=s2, handle=h)
            torch.cuda.synchronize()
            assert K2.cpu().tolist() == K1.cpu().tolist()
            assert np.array_equal(s2.cpu().numpy(), s1.cpu().numpy())
    finally:
        h.close()


def test_noalloc_spa_rejects_inputs_beyond_the_scratch():
    h = api.Handle(0)
    try:
        k, n, r = 128, 40000, 5          # (k + 2) n > 4.19e6 doubles
        B = torch.zeros((k, n), dtype=torch.float32, device=DEV)
        K = torch.full((r,), -7, dtype=torch.int64, device=DEV)
        with pytest.raises(L.CnmfError) as e:
            api.spa(B, r, noalloc=True, K=K, handle=h)
        assert e.value.status == L.CNMF_ENOTSUP and "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert K.cpu().tolist() == [-7] * r      # outputs untouched
    finally:
        h.close()
