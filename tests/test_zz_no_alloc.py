"""The allocation-free adjoint entry point (ljmd_lj_backward_noalloc, partial
sums in the library's static device scratch) against ljmd_lj_backward (the
same kernels with the caller's workspace), called through the C ABI.

Both run the same kernels in the same order, so the outputs must agree bit
for bit.  Two calls in a row on one device, the second with a smaller
system, check that nothing of the first call's scratch contents leaks into
the second; the first call is also checked against the oracle's FP64
adjoint (within 1e-11 normwise, the adjoint's parity bar)."""
import numpy as np
import pytest
import torch

from paper_2508_13523_amd import _lib as L
from paper_2508_13523_amd import api, inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = torch.device("cuda:0")


def run_pair(s, global_format, seed):
    x = torch.tensor(s.x, device=DEV)
    t = torch.tensor(s.types, device=DEV, dtype=torch.int32) if s.ntypes > 1 else None
    prm = api.LJParams.from_system(s)
    nl = api.build_list(x, t, s.box, prm, global_format=global_format)
    g = torch.tensor(np.random.default_rng(seed).normal(size=(s.n, 3)), device=DEV)
    ref = api.lj_backward(x, t, s.box, prm, nl, g)
    T = prm.ntypes
    out = (torch.full((s.n, 3), float("nan"), dtype=torch.float64, device=DEV),
           torch.full((T, T), float("nan"), dtype=torch.float64, device=DEV),
           torch.full((T, T), float("nan"), dtype=torch.float64, device=DEV))
    api.lj_backward_noalloc(x, t, s.box, prm, nl, g, *out)
    torch.cuda.synchronize()
    for a, b in zip(ref, out):
        assert torch.equal(a, b)
    return x.cpu().numpy(), g.cpu().numpy(), out


@pytest.mark.parametrize("fmt", ["tiled", "global"])
def test_noalloc_backward_equals_workspace_entry(oracle, fmt):
    big = inputs.binary_liquid(2000, seed=21)
    small = inputs.binary_liquid(500, seed=22)
    xb, gb, out = run_pair(big, fmt == "global", 23)
    rx, _, _ = oracle.backward_brute(oracle.wrap(big.x, big.box), big.types, big.box, big.eps,
                                     big.sigma, big.rc, gb)
    gx = out[0].cpu().numpy()
    assert np.abs(gx - rx).max() / np.abs(rx).max() < 1e-11
    run_pair(small, fmt == "global", 24)  # second call, smaller input
