"""The allocation-free inference entry point (muffin_cnn_predict_noalloc, workspace in a static
device array) against muffin_cnn_predict on the same inputs: bit-identical outputs over two calls in
a row, the second on a smaller input, plus a case that needs several chunks of the workspace, and
the size limit."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def planes(B, N, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.rand((B, N, N), generator=g, dtype=torch.float32).cuda()


def test_noalloc_inference_equals_predict(lib):
    with lib.Cnn(seed=11) as net:
        for B, N, seed in [(3, 256, 1), (1, 64, 2), (5, 512, 3)]:
            print(f"[no_alloc] B={B} N={N} seed={seed}", flush=True)
            x = planes(B, N, seed)
            ref = net.predict(x).cpu().numpy()
            got = net.predict_noalloc(x).cpu().numpy()
            np.testing.assert_array_equal(got, ref)
            assert np.isfinite(got).all() and np.abs(got).max() > 0


def test_noalloc_inference_rejects_planes_beyond_the_workspace(lib):
    with lib.Cnn(seed=11) as net:
        x = torch.zeros((1, 2048, 2048), dtype=torch.float32, device="cuda")
        with pytest.raises(lib.MuffinError) as e:
            net.predict_noalloc(x)
        assert e.value.code == lib.EINVAL
