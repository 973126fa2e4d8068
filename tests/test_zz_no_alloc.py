"""The no-allocation family entry point against the allocating one.

ranmar_jump_family_noalloc computes what ranmar_jump_family computes (stream
family, Sec. 1 block splitting: start k is the base jumped by k * delta,
Sec. 3.1 and 3.2) with its scratch in a fixed per-device array instead of
device memory allocated per call.  Every call on a device reuses that array,
so the checks run two calls in a row, the second one smaller, and compare
each with ranmar_jump_family bit for bit (integer results: tolerance 0).
"""
import numpy as np
import pytest
import torch

import paper_2512_00093_amd as R
from tests.gpu_util import dev, say, states_t, u32

pytestmark = pytest.mark.gpu


def _family_pair(base, delta, n, variant):
    R.ranmar_tune_set(R.RANMAR_K_FAMILY, variant)
    try:
        ref = R.ranmar_jump_family(base, delta, n)
        got = torch.full((n, 98), -1, dtype=torch.int32, device=dev())
        R.ranmar_jump_family_noalloc(base, delta, n, got)
    finally:
        R.ranmar_tune_set(R.RANMAR_K_FAMILY, -1)
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("variant", [1, 2])
def test_noalloc_family_matches_allocating_entry_point(orc, variant):
    """Product forms (16- and 32-row int8 matrix-core tiles): a 65,536-start
    family (255 shared factors in the fixed array), then a smaller, ragged one
    with 15-digit factors (40,001 starts at spacing 2^104 + 3, the last start
    at ~2^119.3), whose factors overwrite the first call's in the same array."""
    R.ranmar_init()
    base = states_t(orc.state_from_seed(4711))
    for n, delta in ((65_536, 1 << 40), (40_001, (1 << 104) + 3)):
        say(f"noalloc family variant={variant} n={n} delta={delta}")
        ref, got = _family_pair(base, delta, n, variant)
        assert torch.equal(got, ref), (variant, n)
        for k in (0, 1, n // 2, n - 1):
            assert np.array_equal(u32(got[k]), orc.jump(orc.state_from_seed(4711), k * delta)), (variant, n, k)


def test_noalloc_family_small_and_in_place(orc):
    """Below two tiles of starts the product form does not apply and radix
    rounds of table factors serve (no scratch); then a product-form family
    built in place (d_base == d_out) after it."""
    R.ranmar_init()
    seed_state = orc.state_from_seed(31)
    say("noalloc family radix n=600")
    ref, got = _family_pair(states_t(seed_state), (1 << 40) + 7, 600, -1)
    assert torch.equal(got, ref)
    n, delta = 50_000, (1 << 64) + 12345
    say(f"noalloc family in place n={n}")
    fam = torch.zeros((n, 98), dtype=torch.int32, device=dev())
    fam[0] = states_t(seed_state)[0]
    R.ranmar_jump_family_noalloc(fam[:1], delta, n, fam)
    ref = R.ranmar_jump_family(states_t(seed_state), delta, n)
    torch.cuda.synchronize()
    assert torch.equal(fam, ref)


def test_noalloc_family_limits():
    """Beyond the fixed array (n > 2^24) or beyond 128-bit exponents the call
    is refused on the host and nothing is written."""
    R.ranmar_init()
    base = torch.zeros((1, 98), dtype=torch.int32, device=dev())
    out = torch.full((4, 98), 7, dtype=torch.int32, device=dev())
    ptr = lambda t: R._binding._ptr(t)  # noqa: E731
    big = R.RANMAR_NOALLOC_FAMILY_MAX_N + 1
    st = R.lib().ranmar_jump_family_noalloc(ptr(base), R._binding._u128(1), big, ptr(out), R._binding._stream(None))
    assert st == R.RANMAR_EINVAL
    with pytest.raises(R.RanmarError) as ei:
        R.ranmar_jump_family_noalloc(base, 1 << 127, 4, out)
    assert ei.value.status == R.RANMAR_EINVAL
    torch.cuda.synchronize()
    assert bool((out == 7).all())
