"""Served ensembles on the GPU: continuous batching through the C ABI; every
request's result (temperature, VACF) is the same alone and in the mix."""
import numpy as np
import pytest

from paper_2212_11878_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_11878_amd import serve
    return serve


def _small_requests():
    # a burst of small boxes arriving at once, uneven sizes and lengths
    reqs = inputs.served_requests(rate_hz=500, window_s=0.05, seed=5, edge=(6, 20), steps=(20, 120))
    for r in reqs:
        r["arrival"] = 0.0
    return reqs


def test_results_identical_alone_and_in_the_mix(serve):
    print("[case] serve mix", flush=True)
    reqs = _small_requests()
    assert len(reqs) >= 10
    eng = serve.LibraryEngine(hbm_budget=1 << 30, vacf_stride=5)
    summary, mixed = serve.Server(eng, chunk_steps=16).run(reqs)
    eng.close()
    assert summary["completed"] == len(reqs)
    assert summary["max_live"] > 1            # really batched
    by_seed = {d["req"]["seed"]: d for d in mixed}
    for r in reqs[:6]:
        eng = serve.LibraryEngine(hbm_budget=1 << 30, vacf_stride=5)
        _, alone = serve.Server(eng, chunk_steps=16).run([dict(r)])
        eng.close()
        a, m = alone[0], by_seed[r["seed"]]
        assert a["step"] == m["step"] == r["steps"]
        assert a["T"] == m["T"]
        assert np.array_equal(a["vacf"], m["vacf"])


def test_budget_admission_queues_requests(serve):
    print("[case] serve budget", flush=True)
    reqs = _small_requests()
    eng = serve.LibraryEngine(hbm_budget=64 << 20, vacf_stride=5)
    summary, done = serve.Server(eng, chunk_steps=16).run(reqs)
    eng.close()
    assert summary["completed"] == len(reqs)
    assert max(d["queued"] for d in done) > 0.0     # some waited for memory
