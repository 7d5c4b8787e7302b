"""The allocation-free forward pass (cfr_mlp_forward_noalloc) against cfr_mlp_forward, through
the C ABI: the per-layer GEMMs through the shared device array against (for this shape) the
fused three-layer kernel, which computes every element in the same order, so the logits must
agree bit for bit, on two calls in a row (the second with a smaller batch, over the first
call's leftovers in the shared device array), and a batch past the array's limit is refused
with CFR_EINVAL."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_forward_matches_forward():
    import torch
    from paper_2408_14778_amd import CfrError
    from paper_2408_14778_amd.warmstart import WarmStartNet
    F, H, A = 96, 256, 4
    net = WarmStartNet(F, H, A, max_batch=8192, seed=4)
    rng = np.random.default_rng(8)
    for B in (6000, 1234):
        x = torch.from_numpy(rng.standard_normal((B, F)).astype(np.float32)).to("cuda")
        x = x.to(torch.bfloat16)
        ref = net.forward(x)
        out = torch.full((B, A), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(x, out)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), out.cpu().numpy()
        assert np.isfinite(b).all()
        assert np.array_equal(a, b), (B, float(np.abs(a - b).max()))
    big = torch.zeros((16385, F), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(CfrError, match="CFR_EINVAL"):
        net.forward_noalloc(big, torch.empty((16385, A), dtype=torch.float32, device="cuda"))
    net.close()
