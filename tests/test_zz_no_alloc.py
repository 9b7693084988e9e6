"""The allocation-free search entry point (rfr_recombine_dev_noalloc) against
the workspace one (rfr_recombine_dev): same weights and window, bit-identical
pattern sets, over consecutive calls that share the library's fixed device
scratch (the second call smaller than the first, so stale contents of the
first would show)."""
import random
import sys

import pytest

from oracle import rfr_ref as O

pytestmark = pytest.mark.gpu
MASK = (1 << 64) - 1


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2410_15880_amd as R
    R.lib()
    return R


def planted(rng, n, rel=3):
    """Random 64-bit weights with a few subset relations planted inside the window."""
    w = [rng.getrandbits(64) for _ in range(n)]
    for _ in range(rel):
        idx = rng.sample(range(n - 1), rng.randint(2, 8))
        tot = sum(w[i] for i in idx[:-1])
        w[idx[-1]] = (-tot - rng.randint(0, n)) & MASK
    return w


def noalloc(R, w, t_lo, t_hi, cap=4096):
    import torch
    cand = torch.empty(2 * cap, dtype=torch.int64, device="cuda")
    count = torch.empty(1, dtype=torch.int64, device="cuda")
    R.recombine_dev_noalloc(w, t_lo, t_hi, cand, count)
    torch.cuda.synchronize()
    return R.read_patterns(len(w), cand, count)


def test_noalloc_matches_workspace_entry_on_consecutive_calls(R):
    rng = random.Random(2024)
    assert R.lib().rfr_recombine_noalloc_scratch_bytes() == 64 << 20
    # n = 46: halves of 2^23 and 2^22 keys, half A streamed in chunks through
    # the scratch; then n = 33 (one pass, much smaller tables) and n = 17
    # (the one-workgroup search)
    for n, t_lo, t_hi in [(46, 60, 8), (33, 40, 5), (17, 20, 3)]:
        w = planted(rng, n)
        say("noalloc n=%d" % n)
        got = noalloc(R, w, t_lo, t_hi)
        want = R.recombine_dev(w, t_lo, t_hi)
        assert got == want, (n, len(got), len(want))
        assert len(got) >= 1
        if n <= 23:
            assert got == O.search_brute(w, t_lo, t_hi)


def test_noalloc_rejects_too_many_elements(R):
    rng = random.Random(7)
    w = [rng.getrandbits(64) for _ in range(47)]
    with pytest.raises(R.RFRError) as e:
        noalloc(R, w, 10, 10)
    assert e.value.status == -3  # RFR_ENOMEM


def test_noalloc_overflow_then_clean_call(R):
    # all-zero weights flood the candidate buffer (every pattern is in the
    # window): the overflow is reported, and the next call on the same scratch
    # is exact again
    w = [0] * 30
    with pytest.raises(R.RFRError) as e:
        noalloc(R, w, 40, 5, cap=64)
    assert e.value.status == -6
    rng = random.Random(11)
    w = planted(rng, 30)
    assert noalloc(R, w, 40, 5) == R.recombine_dev(w, 40, 5)
