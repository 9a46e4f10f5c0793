"""The direct correlator's entry point that allocates nothing, through the C ABI: the same visibilities as
omni_direct_correlate, bit for bit (both are exact integer sums rounded once to float32), on two calls in a row
sharing the library's fixed device scratch, the second with a smaller input (fewer antennas, channels and
samples, so stale half-sums of the first call would show)."""

import math
import sys

import pytest
import torch

import paper_0909_0001_amd as omni
import skysim

pytestmark = pytest.mark.gpu


def _raw(dtype, T, F, N, seed):
    gen = torch.Generator().manual_seed(seed)
    if dtype == "ci8":
        return torch.randint(-128, 128, (T, F, N, 2), generator=gen, dtype=torch.int16).to(torch.int8)
    re = torch.randint(-8, 8, (T, F, N), generator=gen, dtype=torch.int16)
    im = torch.randint(-8, 8, (T, F, N), generator=gen, dtype=torch.int16)
    return skysim.pack_ci4(re, im)


@pytest.mark.parametrize("dtype", ["ci8", "ci4"])
def test_noalloc_matches_direct_correlate(dtype):
    cases = [([[4, 8], [4, 8]], 3, 70), ([[16, 16]], 2, 33)]  # 1024 then 256 antennas
    for level_dims, F, T in cases:
        N = math.prod(v for ld in level_dims for v in ld)
        print("noalloc", dtype, level_dims, "F", F, "T", T, file=sys.stderr, flush=True)
        raw = _raw(dtype, T, F, N, N + T).cuda()
        plan = omni.Plan(level_dims, None, F, dtype, "fp32")
        want = plan.direct_correlate(raw)
        got = torch.full_like(want, float("nan"))
        plan.direct_correlate_noalloc(raw, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), level_dims


def test_noalloc_refuses_oversized_call():
    """More half-sums than the fixed scratch holds is refused before any launch (8x8 tiles of 8x8, 96 channels)."""
    plan = omni.Plan([[8, 8], [8, 8]], None, 96, "ci8", "fp32")
    raw = torch.zeros((1, 96, 4096, 2), dtype=torch.int8, device="cuda")
    out = torch.empty(plan.vis_shape(), dtype=torch.complex64, device="cuda")
    with pytest.raises(omni.OmniError, match="fixed scratch") as ei:
        plan.direct_correlate_noalloc(raw, out)
    assert omni.STATUS[ei.value.code] == "OMNI_E_NOMEM"
