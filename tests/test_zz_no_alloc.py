"""pt_selftest_noalloc, the entry point for callers that cannot allocate
device memory, against pt_selftest (same kernels, staging in a fixed device
array instead of per-call buffers): bit-identical outputs on two calls in a
row, the second with a smaller input, for every op; sizes beyond the array
fail cleanly and leave the entry point usable."""
import math

import numpy as np
import pytest

from paper_1107_3490_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_3490_amd import pt
    pt.lib()  # raises if the HIP library is missing: no fallback
    yield


def _inputs(op, n, rng):
    from paper_1107_3490_amd import pt
    if op == pt.OP_PHILOX:
        return rng.integers(0, 2 ** 32, size=4 * n).astype(np.float64), np.array([12345.0, 678.0])
    if op == pt.OP_MOVE32:
        x = np.zeros((n, pt.MOVE_ITEM))
        x[:, 0:3 * 512:3] = 1.0e30
        for i in range(n):
            nb = int(rng.integers(2, 513))
            x[i, :3 * nb] = I.random_walk(nb, rng).ravel()
            x[i, 3 * 512:3 * 512 + 5] = [nb, int(rng.integers(0, nb)), *((rng.random(3) - 0.5) * 0.2)]
        return x.ravel(), None
    if op == pt.OP_LJ32:
        r = rng.uniform(0.3, 3.0, n)
        phi = rng.uniform(0, 2 * math.pi, n)
        return r * np.cos(phi), r * np.sin(phi)
    x = rng.uniform(0.1, 3.0, n)
    if op in (pt.OP_WAVE64, pt.OP_WAVE32):
        x = rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))
    y = rng.uniform(0.5, 2.0, n) if op == pt.OP_DIV else None
    return x, y


# (op, n of the first call, n of the second): the first call fills most of
# the staging array, the second, smaller one must not see its leftovers.
CASES = [(0, 700000, 1000), (1, 500000, 333), (2, 600000, 77), (3, 300000, 5000), (4, 600000, 1),
         (5, 500000, 999), (6, 200000, 3), (7, 64 * 10000, 64), (8, 64 * 10000, 128), (9, 1300, 7)]


@pytest.mark.parametrize("op,n1,n2", CASES)
def test_noalloc_equals_selftest_on_two_calls(op, n1, n2):
    from paper_1107_3490_amd import pt
    m = I.model_params()
    rng = np.random.default_rng(500 + op)
    print(f"\n[case] no-alloc op {op}: n = {n1} then {n2}", flush=True)
    for n in (n1, n2):
        x, y = _inputs(op, n, rng)
        want = pt.pt_selftest(m, op, x, y)
        got = pt.pt_selftest_noalloc(m, op, x, y)
        assert got.shape == want.shape
        same = (got == want) | (np.isnan(got) & np.isnan(want))
        assert np.all(same), (op, n, np.flatnonzero(~same)[:5])


def test_noalloc_rejects_sizes_beyond_its_array():
    from paper_1107_3490_amd import pt
    m = I.model_params()
    limit = 1 << 21
    x = np.ones(limit // 2 + 1)              # op 0: n + n doubles > limit
    with pytest.raises(RuntimeError, match="no-allocation buffer"):
        pt.pt_selftest_noalloc(m, pt.OP_SQRT, x)
    # still usable, and still equal to pt_selftest, after the refusal
    x = np.linspace(0.5, 4.0, 4096)
    assert np.array_equal(pt.pt_selftest_noalloc(m, pt.OP_SQRT, x), pt.pt_selftest(m, pt.OP_SQRT, x))
