"""The plan tuner end to end on the GPU (row T): a small tuning run times
whole solves through the C ABI, writes the plan cache, and a handle created
with leaf = 0 / crossover = 0 picks the measured winner from that file and
solves to the float64 bar against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL64 = 1e-11


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_11593_amd import binding

    binding.lib()
    return torch


def test_tuned_plan_is_read_back_and_solves(torch_cuda, orc, tmp_path, monkeypatch):
    from paper_1710_11593_amd import binding, tune
    from paper_1710_11593_amd import workloads as wl

    path = tmp_path / "plan.json"
    monkeypatch.setenv("FRACSOLVE_TUNE_CACHE", str(path))
    monkeypatch.delenv("FRACSOLVE_TUNE", raising=False)
    lines = []
    plan = tune.tune(N=1024, reps=1, precisions=("fp64",), buckets=(64,), leaves=(4, 8),
                     crossovers=(-1, 16, 64), log=lines.append)
    timed = {k: v for k, v in plan["timings_ms"].items()}
    assert len(timed) == 6 and all(v is not None and v > 0 for v in timed.values()), timed
    (e,) = [x for x in plan["entries"] if x["m_max"] == 64]
    assert abs(e["ms"] - min(timed.values())) <= 1e-4  # the file keeps 4 decimals
    tune.write(plan, str(path))
    leaf, cross, src = binding.plan([dict(gamma=0.4, M=50, N=700)])
    assert (leaf, cross, src) == (e["leaf"], e["crossover"], "cache")

    M, N, gamma = 50, 700, 0.4
    rng = np.random.default_rng(7)
    x, _, _, _ = wl.grid(M, N)
    f = np.outer(np.linspace(1.0, 2.0, N), np.sin(np.pi * x)) + 0.2 * rng.standard_normal((N, M))
    s = binding.Solver([dict(gamma=gamma, M=M, N=N)])
    s.set_timing(True)
    u = s.solve([torch_cuda.from_numpy(f).cuda()])[0].cpu().numpy()
    st = s.stats()
    s.close()
    assert (st["leaf"], st["crossover"]) == (e["leaf"], e["crossover"])
    ref = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, f)
    assert np.max(np.abs(u - ref)) / np.max(np.abs(ref)) <= TOL64
