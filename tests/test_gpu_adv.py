"""GPU parity of the advection equations (Schemes 2 and 3, equation =
FRACSOLVE_ADVECTION) against the oracle's time stepping.

Bar: max-norm relative error <= 1e-11 (float64; where the oracle's own
float64 error exceeds that, within the number of recursion levels times the
oracle's distance to an extended-precision solve), on sizes that span several
leaves and levels with ragged tails, through the dense and the FFT level
routes, in batches that mix both schemes; and the paper's Tables 5 and 7
recomputed from the GPU solutions to the printed digits.
"""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-11
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_11593_amd import binding

    binding.lib()
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def relerr(x, ref):
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def case(gamma, M, N, seed=0):
    rng = np.random.default_rng(seed)
    h = 1.0 / (M + 1)
    x = h * np.arange(1, M + 1)
    t = np.arange(1, N + 1) / N
    f = np.outer(1 + t ** 2, np.sin(np.pi * x)) + 0.2 * rng.standard_normal((N, M))
    u0 = np.sin(np.pi * x) * x
    phi = np.cos(np.pi * x) * x if gamma > 1 else None
    return f, u0, phi


def assert_parity(u, ref, gamma, M, N, f, u0, phi):
    """<= 1e-11 against the oracle; where the oracle's own float64 error
    exceeds that (diffusion-wave data amplify rounding), the floor regime's
    checks: forward errors against an extended-precision solve <= 1e-8 and
    the GPU's backward error at most 8 ulp or twice the oracle's."""
    e = relerr(u, ref)
    if e <= TOL:
        return
    import oracle
    from tests import ext_reference
    from tests.test_gpu_parity import gpu_weights

    ext = np.asarray(ext_reference.solve_adv(gamma, M, N, f, u0, phi), dtype=np.float64)
    e_gpu, e_orc = relerr(u, ext), relerr(ref, ext)
    eta_gpu = ext_reference.backward_adv(gpu_weights(gamma, N), gamma, M, N, f, u, u0, phi)
    eta_orc = ext_reference.backward_adv(oracle.weights(gamma, 1.0, N), gamma, M, N, f, ref, u0, phi)
    print("  floor: vs extended gpu %.2e oracle %.2e; backward error gpu %.2f oracle %.2f ulp"
          % (e_gpu, e_orc, eta_gpu / ext_reference.EPS, eta_orc / ext_reference.EPS), flush=True)
    ext_reference.assert_floor_parity(e, e_gpu, e_orc, eta_gpu, eta_orc, TOL)


def gpu_solve(torch, probs, fields, **opts):
    from paper_1710_11593_amd import binding

    s = binding.Solver([dict(gamma=g, M=M, N=N) for g, M, N in probs], equation="advection", **opts)
    f = [dev(torch, c[0]) for c in fields]
    u0 = [dev(torch, c[1]) for c in fields]
    phi = [dev(torch, c[2]) if c[2] is not None else None for c in fields]
    us = s.solve(f, u0, phi)
    torch.cuda.synchronize()
    out = [u.cpu().numpy() for u in us]
    s.close()
    return out


@pytest.mark.parametrize("gamma", [0.1, 0.6, 1.3, 1.9])
@pytest.mark.parametrize("M,N", [(1, 10), (31, 32), (100, 77), (255, 256), (1000, 300), (4096, 64), (2047, 129)])
def test_parity_with_the_oracle(torch_cuda, orc, gamma, M, N):
    f, u0, phi = case(gamma, M, N, seed=M + N)
    (u,) = gpu_solve(torch_cuda, [(gamma, M, N)], [(f, u0, phi)])
    ref = orc.solve_adv(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    print("adv", gamma, M, N, relerr(u, ref), flush=True)
    assert_parity(u, ref, gamma, M, N, f, u0, phi)


@pytest.mark.parametrize("gamma", [0.4, 1.6])
@pytest.mark.parametrize("opts", [dict(crossover=-1), dict(leaf=4), dict(crossover=16, leaf=4)])
def test_level_routes_and_leaf_sizes(torch_cuda, orc, gamma, opts):
    M, N = 130, 333
    f, u0, phi = case(gamma, M, N, seed=7)
    (u,) = gpu_solve(torch_cuda, [(gamma, M, N)], [(f, u0, phi)], **opts)
    ref = orc.solve_adv(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    assert_parity(u, ref, gamma, M, N, f, u0, phi)


def test_multipass_levels(torch_cuda, orc):
    # N > 8192 pads to 16384 or more: the largest levels take the multi-pass
    # FFT route (N = 9000 for the diffusion-wave case keeps its
    # extended-precision check short)
    for gamma, N in ((0.5, 20000), (1.5, 9000)):
        M = 8
        f, u0, phi = case(gamma, M, N, seed=3)
        (u,) = gpu_solve(torch_cuda, [(gamma, M, N)], [(f, u0, phi)])
        ref = orc.solve_adv(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
        assert_parity(u, ref, gamma, M, N, f, u0, phi)


def test_batch_mixing_both_schemes(torch_cuda, orc):
    probs = [(0.3, 64, 100), (1.4, 200, 64), (0.8, 1, 33), (1.7, 513, 40), (0.2, 37, 130)]
    fields = [case(g, M, N, seed=k) for k, (g, M, N) in enumerate(probs)]
    us = gpu_solve(torch_cuda, probs, fields)
    for (g, M, N), (f, u0, phi), u in zip(probs, fields, us):
        ref = orc.solve_adv(g, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
        assert_parity(u, ref, g, M, N, f, u0, phi)


def test_in_place_and_zero_data(torch_cuda, orc):
    from paper_1710_11593_amd import binding

    for gamma in (0.5, 1.5):
        M, N = 50, 60
        f, u0, phi = case(gamma, M, N, seed=11)
        s = binding.Solver([dict(gamma=gamma, M=M, N=N)], equation="advection")
        fd = dev(torch_cuda, f)
        s.solve([fd], [dev(torch_cuda, u0)], [dev(torch_cuda, phi)] if phi is not None else None, out=[fd])
        z = s.solve([dev(torch_cuda, np.zeros((N, M)))])[0]
        torch_cuda.cuda.synchronize()
        ref = orc.solve_adv(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
        assert relerr(fd.cpu().numpy(), ref) <= TOL
        assert not z.cpu().numpy().any()
        s.close()


def read_table(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        misprint = parts[3].split("=")[1] if len(parts) > 3 else None
        rows.append((float(parts[0]), int(parts[1]), parts[2], misprint))
    return rows


def within_printed(err, printed):
    target = float(printed)
    e = math.floor(math.log10(target))
    return abs(err - target) <= 1.0001 * 10 ** (e - 4)


def test_tables_5_and_7_from_gpu_solutions(torch_cuda):
    for gamma, k, printed, _ in read_table("table5.txt"):
        Mp, N = 2 ** k, 2 ** 10
        h = 1.0 / Mp
        x = h * np.arange(1, Mp)
        t = np.arange(1, N + 1) / N
        xm = x - h / 2
        f = (np.outer(t ** (1 - gamma) / math.gamma(2 - gamma), np.sin(np.pi * xm))
             + np.outer(np.pi * t, np.cos(np.pi * xm)))
        (u,) = gpu_solve(torch_cuda, [(gamma, Mp - 1, N)], [(f, np.zeros(Mp - 1), None)])
        err = math.sqrt(h * np.sum((u[-1] - np.sin(np.pi * x)) ** 2))
        assert within_printed(10.0 * err, printed), (gamma, k, err, printed)
    for gamma, k, printed, misprint in read_table("table7.txt"):
        Mp = N = 2 ** k
        h = 1.0 / Mp
        x = h * np.arange(1, Mp)
        th = (np.arange(1, N + 1) - 0.5) / N
        f = (np.outer(6 * th ** (3 - gamma) / math.gamma(4 - gamma), x - x * x)
             + np.outer(th ** 3, 1 - 2 * x))
        (u,) = gpu_solve(torch_cuda, [(gamma, Mp - 1, N)], [(f, np.zeros(Mp - 1), None)])
        err = math.sqrt(h * np.sum((u[-1] - x * (1 - x)) ** 2))
        assert within_printed(err, misprint or printed), (gamma, k, err, printed)


def test_unsupported_calls_are_rejected(torch_cuda):
    from paper_1710_11593_amd import binding

    with pytest.raises(binding.FracsolveError, match="float64"):
        binding.Solver([dict(gamma=0.5, M=8, N=8)], equation="advection", precision="fp32", refine_steps=1)
    s = binding.Solver([dict(gamma=0.5, M=8, N=8)], equation="advection")
    x = dev(torch_cuda, np.ones((8, 8)))
    for call in (lambda: s.apply([x]), lambda: s.adjoint([x], [x]), lambda: s.gmres([x])):
        with pytest.raises(binding.FracsolveError, match="advection"):
            call()
    s.close()
