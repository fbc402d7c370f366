"""GPU tests of the two measurement aids of the C ABI: the event log that
samples the solvers' dense products with HIP events (ccg_set_event_log), and
the read-stream pass (ccg_read_stream)."""
import numpy as np
import pytest

from gpu_util import dev
from paper_1208_4869_amd import ccg, inputs

pytestmark = pytest.mark.gpu


def test_event_log_samples_the_products_and_changes_nothing():
    """With a log attached the solve gives the same bits; every counted
    product of the chosen kinds is sampled at stride 1, every third at stride
    3; the v = A p products of a BiCGSTAB solve number at least its
    iterations plus its confirmations; other kinds are not counted; after
    detaching nothing more is recorded."""
    import torch
    A, _, y = inputs.dense_system(300, 11)
    Ad, yd = dev(A), dev(y)
    x0 = torch.empty_like(yd)
    r0 = ccg.ccg_bicgstab_ex(Ad, yd, x0, 1e-10, 1000, flags=ccg.X0_ZERO)
    log = ccg.EventLog(64, stride=1, roles=ccg.PROD_V)
    x1 = torch.empty_like(yd)
    with log:
        r1 = ccg.ccg_bicgstab_ex(Ad, yd, x1, 1e-10, 1000, flags=ccg.X0_ZERO)
    torch.cuda.synchronize()
    assert torch.equal(x0, x1) and r0 == r1
    assert log.count == log.seen >= r1.iters + r1.confirms
    d = log.durations()
    assert len(d) == log.count and all(t > 0 for t in d)
    # stride 3: every third counted launch
    log3 = ccg.EventLog(64, stride=3, roles=ccg.PROD_V)
    with log3:
        ccg.ccg_bicgstab_ex(Ad, yd, x1, 1e-10, 1000, flags=ccg.X0_ZERO)
    assert log3.seen == log.seen and log3.count == (log3.seen + 2) // 3
    # CGNR's products are not of kind v: none counted
    logc = ccg.EventLog(8, stride=1, roles=ccg.PROD_V)
    with logc:
        ccg.ccg_cgnr_ex(Ad, yd, x1, 1e-10, 1000, flags=ccg.X0_ZERO)
    assert logc.seen == 0 and logc.count == 0
    # detached: nothing more
    ccg.ccg_bicgstab_ex(Ad, yd, x1, 1e-10, 1000, flags=ccg.X0_ZERO)
    assert log.count == log.seen
    # capacity bounds the pairs
    small = ccg.EventLog(2, stride=1, roles=0)
    with small:
        ccg.ccg_bicgstab_ex(Ad, yd, x1, 1e-10, 1000, flags=ccg.X0_ZERO)
    assert small.count == 2 and small.seen >= r1.matvecs


@pytest.mark.parametrize("nbytes", [16, 4096, 262144, 262144 + 48, 3 * 262144 + 1024])
def test_read_stream_sums_every_slab(nbytes):
    """Each block's sum is the sum of its slab of 256 KiB (ragged last slab
    included), so every byte was read."""
    import torch
    n16 = nbytes // 16
    rng = np.random.default_rng(nbytes)
    vals = (rng.integers(-4, 5, n16) + 1j * rng.integers(-4, 5, n16)).astype(np.complex128)
    src = dev(vals)
    out = ccg.ccg_read_stream(src)
    torch.cuda.synchronize()
    slab = ccg.READ_STREAM_SLAB // 16
    nb = (n16 + slab - 1) // slab
    got = out.cpu().numpy()[:nb]
    want = np.array([vals[b * slab:(b + 1) * slab].sum() for b in range(nb)])
    assert np.array_equal(got, want)  # small integers: exact in any order
