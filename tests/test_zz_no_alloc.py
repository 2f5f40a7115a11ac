"""The allocation-free residual entry point (awe_residual_noalloc, static device scratch)
against awe_residual (caller workspace), through the C ABI: bitwise equal residual and
misfit on two calls in a row, the second one smaller, with nothing allocated by the call."""
import numpy as np
import pytest
import torch

import paper_2304_05592_amd as A

pytestmark = pytest.mark.gpu


def test_residual_noalloc_matches_residual_on_two_calls():
    rng = np.random.default_rng(11)
    for n in (3_000_017, 100_003):      # the second call reduces fewer values
        a = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
        b = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
        r_ref, loss_ref = A.residual(a, b)
        r = torch.empty_like(a)
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        before = torch.cuda.memory_stats()["allocation.all.allocated"]
        A.residual_noalloc(a, b, r, loss)
        after = torch.cuda.memory_stats()["allocation.all.allocated"]
        torch.cuda.synchronize()
        assert after == before
        assert torch.equal(r, r_ref)
        assert loss.item() == loss_ref.item()
        ref = 0.5 * np.sum((a.cpu().numpy() - b.cpu().numpy()).astype(np.float64) ** 2)
        assert abs(loss.item() - ref) <= 1e-12 * ref
        print(f"n={n}: loss {loss.item():.9e} (reference {ref:.9e})", flush=True)
