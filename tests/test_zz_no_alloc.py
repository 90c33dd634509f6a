"""mpcd_moments_noalloc (the entry point for callers that cannot allocate)
against mpcd_moments on the same device arrays, through the C ABI: two calls
in a row, the second on fewer particles, each bit for bit equal to the
allocating call."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_equals_allocating_on_two_calls():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_11878_amd import mpcd
    noalloc = mpcd.mpcd_moments_noalloc
    stream = torch.cuda.current_stream().cuda_stream
    for n, masses in ((3_000_001, True), (100_003, False)):   # the second call is smaller
        print("[case] noalloc n=%d masses=%s" % (n, masses), flush=True)
        rng = np.random.default_rng(n)
        v = [torch.from_numpy(rng.normal(size=n).astype(np.float32)).cuda() for _ in range(3)]
        m = torch.from_numpy(rng.uniform(0.5, 2.0, n).astype(np.float32)).cuda() if masses else None
        mp_ = m.data_ptr() if m is not None else None
        out_a = torch.zeros(5, dtype=torch.float64, device="cuda")
        out_b = torch.full((5,), -1.0, dtype=torch.float64, device="cuda")
        assert mpcd.mpcd_moments(v[0].data_ptr(), v[1].data_ptr(), v[2].data_ptr(), mp_ or 0, n,
                                 out_a.data_ptr(), stream) == mpcd.MPCD_OK
        assert noalloc(v[0].data_ptr(), v[1].data_ptr(), v[2].data_ptr(), mp_ or 0, n, out_b.data_ptr(),
                       stream) == mpcd.MPCD_OK
        torch.cuda.synchronize()
        a, b = out_a.cpu().numpy(), out_b.cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (a, b)
        assert a[4] == 0
    # beyond the workspace: refused before any launch
    big = (1 << 28) + 1
    assert noalloc(v[0].data_ptr(), v[1].data_ptr(), v[2].data_ptr(), 0, big, out_b.data_ptr(),
                   stream) == mpcd.MPCD_EINVAL
    assert noalloc(0, 0, 0, 0, 5, out_b.data_ptr(), stream) == mpcd.MPCD_EINVAL
