"""lpt_radix_sort_static, the allocation-free entry point, against
lpt_radix_sort (the allocating one) and a stable argsort, through the C ABI:
two calls in a row, the second smaller (the scratch keeps the first call's
contents), the largest size it accepts, a single key, and the size limit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2607_17836_amd import lpt

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _keys(count, bits, seed):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 1 << bits, count, dtype=np.uint64).astype(np.uint32)
    keys[: count // 3] = keys[0]   # heavy ties: stability matters
    return keys


def test_static_sort_matches_the_allocating_sort_on_two_calls():
    tr = lpt.Tracker(16, "fp64")
    for count, bits, seed in ((lpt.STATIC_SORT_MAX, 24, 1), (100003, 13, 2), (4097, 32, 3)):
        say(f"static sort count={count} bits={bits}")
        keys = _keys(count, bits, seed)
        dk = torch.from_numpy(keys.view(np.int32)).cuda()
        sk, perm = tr.radix_sort_static(dk, bits)
        torch.cuda.synchronize()
        ak, aperm = tr.radix_sort(dk, bits)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(perm.cpu().numpy(), aperm.cpu().numpy())
        np.testing.assert_array_equal(sk.cpu().numpy(), ak.cpu().numpy())
        expect = oracle.sort_permutation(keys)
        np.testing.assert_array_equal(perm.cpu().numpy().view(np.uint32), expect.astype(np.uint32))
        np.testing.assert_array_equal(sk.cpu().numpy().view(np.uint32), keys[expect])
    tr.close()


def test_static_sort_edge_cases_and_limit():
    tr = lpt.Tracker(16, "fp64")
    one = torch.tensor([12345], dtype=torch.int32, device="cuda")
    sk, perm = tr.radix_sort_static(one, 16)
    torch.cuda.synchronize()
    assert sk.item() == 12345 and perm.item() == 0
    big = torch.zeros(lpt.STATIC_SORT_MAX + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(lpt.LptError) as e:
        tr.radix_sort_static(big, 8)
    assert e.value.status == lpt.E_ARG
    assert "at most" in str(e.value)
    tr.close()
