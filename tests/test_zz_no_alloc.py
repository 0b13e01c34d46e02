"""The no-allocation Scheme 1 entry point (fracsolve_ode_cg_noalloc) against
the allocating one (fracsolve_ode_cg) through the C ABI: three calls in a
row on the same fixed workspace, the largest size it accepts first, then
smaller ones, so that each call starts from the contents the previous call
left behind."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_11593_amd import binding

    binding.lib()
    return torch


def test_noalloc_matches_the_allocating_entry_point(torch_cuda):
    from paper_1710_11593_amd import binding

    torch = torch_cuda
    gamma = 0.5
    for N, rtol in ((2 ** 19 + 1, 1e-10), (4097, 1e-12), (1025, 1e-12)):
        t = np.arange(1, N) / N
        f = torch.from_numpy(np.sin(np.pi * t) + t * (1 - t)).cuda()
        print("noalloc: N = %d" % N, flush=True)
        ref, iref, href = binding.ode_cg(gamma, N, f, rtol=rtol, max_iters=5000, hist_cap=64)
        out = torch.full_like(f, float("nan"))
        u, info, hist = binding.ode_cg(gamma, N, f, out=out, rtol=rtol, max_iters=5000, hist_cap=64,
                                       noalloc=True)
        torch.cuda.synchronize()
        assert u.data_ptr() == out.data_ptr()
        assert info["converged"] and info["iterations"] == iref["iterations"], (info, iref)
        err = float((u - ref).abs().max() / ref.abs().max())
        assert err <= 1e-13, err
        assert np.allclose(hist, href, rtol=1e-12, atol=0.0)
        assert abs(info["relres"] - iref["relres"]) <= 1e-6 * iref["relres"] + 1e-300


def test_noalloc_rejects_sizes_beyond_its_workspace(torch_cuda):
    from paper_1710_11593_amd import binding

    torch = torch_cuda
    N = 2 ** 19 + 2
    f = torch.ones(N - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(binding.FracsolveError, match="fixed workspace"):
        binding.ode_cg(0.5, N, f, noalloc=True)
    with pytest.raises(binding.FracsolveError, match="fixed history"):
        binding.ode_cg(0.5, 1025, f[:1024], noalloc=True, hist_cap=65537)
