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


def test_cancel_in_flight_leaves_the_others_unchanged(serve):
    """One request is cancelled while its box is live, with steps of it still
    queued on the device: its memory is released at once, and every other
    request's temperature and VACF equal those of the uncancelled mix bit for
    bit."""
    print("[case] serve cancel", flush=True)
    reqs = _small_requests()
    victim = max(reqs, key=lambda r: r["steps"])
    eng = serve.LibraryEngine(hbm_budget=1 << 30, vacf_stride=5)
    _, full = serve.Server(eng, chunk_steps=16).run([dict(r) for r in reqs])
    eng.close()

    eng = serve.LibraryEngine(hbm_budget=1 << 30, vacf_stride=5)
    srv = serve.Server(eng, chunk_steps=16)
    calls = [0]
    real_step = eng.step

    def step(n):       # cancel after the third chunk is queued (no sync in between)
        real_step(n)
        calls[0] += 1
        if calls[0] == 3:
            srv.cancel(victim["seed"])
    eng.step = step
    summary, part = srv.run([dict(r) for r in reqs])
    eng.close()
    assert summary["cancelled"] == 1 and summary["completed"] == len(reqs) - 1
    a = {d["req"]["seed"]: d for d in full}
    b = {d["req"]["seed"]: d for d in part}
    assert b[victim["seed"]]["status"] == "cancelled"
    assert 0 < b[victim["seed"]]["step"] < victim["steps"]
    for r in reqs:
        if r["seed"] == victim["seed"]:
            continue
        assert b[r["seed"]]["step"] == a[r["seed"]]["step"] == r["steps"]
        assert b[r["seed"]]["T"] == a[r["seed"]]["T"]
        assert np.array_equal(b[r["seed"]]["vacf"], a[r["seed"]]["vacf"])
