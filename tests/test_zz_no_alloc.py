"""The allocation-free FP32 network forward (rbf_mlp_forward_static, through the C ABI)
against the allocating one (rbf_mlp_forward, precision F32): same kernels, so the outputs
agree bit for bit, on two calls in a row, the second with fewer rows."""
import ctypes

import numpy as np
import pytest

from oracle import precond as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _params(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in P.LAYERS:
        parts.append(rng.normal(0, np.sqrt(2.0 / i), (o, i)).ravel())
        parts.append(rng.normal(0, 0.05, o))
    return np.concatenate(parts).astype(np.float32)


def test_static_forward_equals_allocating_forward():
    from paper_1606_07652_amd import _lib as L
    from paper_1606_07652_amd.pc import Mlp
    m = Mlp(_params(71))
    rng = np.random.default_rng(72)
    for rows in (L.RBF_MLP_STATIC_MAX_ROWS, 1000):      # the maximum, then a smaller call
        print(f"[no_alloc] rows={rows}", flush=True)
        x = torch.as_tensor(rng.normal(0, 1, (rows, 64)).astype(np.float32), device="cuda")
        ref = m.forward(x, "f32")
        out = torch.full((rows, 64), float("nan"), dtype=torch.float32, device="cuda")
        m.forward_static(x, out)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), f"max |diff| {np.abs(a - b).max():.3e}"
        assert np.abs(b).max() > 0
    m.close()


def test_static_forward_rejects_too_many_rows():
    from paper_1606_07652_amd import _lib as L
    from paper_1606_07652_amd.pc import Mlp
    m = Mlp(_params(73))
    rows = L.RBF_MLP_STATIC_MAX_ROWS + 1
    x = torch.zeros((rows, 64), dtype=torch.float32, device="cuda")
    y = torch.zeros((rows, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(L.RbfError) as e:
        m.forward_static(x, y)
    assert "static workspace" in str(e.value)
    # zero rows is a no-op
    lib = L.load()
    assert lib.rbf_mlp_forward_static(m._h, None, 0, None, ctypes.c_void_p(0)) == L.RBF_OK
    m.close()
