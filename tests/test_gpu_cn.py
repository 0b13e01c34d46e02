"""GPU parity of the diffusion-wave variant with the spatial term averaged
over t_n and t_{n-1} (equation = FRACSOLVE_DIFFUSION_CN) against the
oracle's time stepping, apply and single-mode recurrence.

Bar: max-norm relative error <= 1e-11 (float64; where the oracle's own
float64 error exceeds that, the GPU's distance to an extended-precision
solve must stay within the number of recursion levels times the oracle's
distance to it), over sizes that span
several leaves and levels, both column orders of the leaf, both level
routes, batches, the operator apply, the adjoint (dot-product identity) and
GMRES.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-11


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


def assert_parity(u, ref, gamma, M, N, f, u0, phi):
    """<= 1e-11 against the oracle; where the oracle's own float64 error
    exceeds that (Thomas' rounding of a_0 + e next to e at large M), the floor
    regime's checks: forward errors against an extended-precision solve
    <= 1e-8 and the GPU's backward error at most 8 ulp or twice the
    oracle's."""
    e = relerr(u, ref)
    if e <= TOL:
        return
    import oracle
    from tests import ext_reference
    from tests.test_gpu_parity import gpu_weights

    ext = np.asarray(ext_reference.solve_cn(gamma, M, N, f, u0, phi), dtype=np.float64)
    e_gpu, e_orc = relerr(u, ext), relerr(ref, ext)
    eta_gpu = ext_reference.backward(gpu_weights(gamma, N), M, N, f, u, u0, phi, kind="cn")
    eta_orc = ext_reference.backward(oracle.weights(gamma, 1.0, N), M, N, f, ref, u0, phi, kind="cn")
    print("  floor: vs extended gpu %.2e oracle %.2e; backward error gpu %.2f oracle %.2f ulp"
          % (e_gpu, e_orc, eta_gpu / ext_reference.EPS, eta_orc / ext_reference.EPS), flush=True)
    ext_reference.assert_floor_parity(e, e_gpu, e_orc, eta_gpu, eta_orc, TOL)


def case(gamma, M, N, seed=0):
    rng = np.random.default_rng(seed)
    x = np.arange(1, M + 1) / (M + 1)
    th = (np.arange(1, N + 1) - 0.5) / N
    f = np.outer(1 + th ** 2, np.sin(np.pi * x)) + 0.2 * rng.standard_normal((N, M))
    return f, np.sin(2 * np.pi * x), np.cos(np.pi * x) * np.sin(np.pi * x)


def solver(probs, **opts):
    from paper_1710_11593_amd import binding

    return binding.Solver([dict(gamma=g, M=M, N=N) for g, M, N in probs], equation="diffusion_cn", **opts)


def gpu_solve(torch, probs, fields, **opts):
    s = solver(probs, **opts)
    us = s.solve([dev(torch, c[0]) for c in fields], [dev(torch, c[1]) for c in fields],
                 [dev(torch, c[2]) for c in fields])
    torch.cuda.synchronize()
    out = [u.cpu().numpy() for u in us]
    s.close()
    return out


@pytest.mark.parametrize("gamma", [1.1, 1.5, 1.9])
@pytest.mark.parametrize("M,N", [(1, 9), (31, 32), (64, 100), (256, 300), (1000, 200), (2048, 129), (4096, 64),
                                 (4095, 70)])
def test_parity_with_the_oracle(torch_cuda, orc, gamma, M, N):
    f, u0, phi = case(gamma, M, N, seed=M + N)
    (u,) = gpu_solve(torch_cuda, [(gamma, M, N)], [(f, u0, phi)])
    ref = orc.solve_cn(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    print("cn", gamma, M, N, relerr(u, ref), flush=True)
    assert_parity(u, ref, gamma, M, N, f, u0, phi)


@pytest.mark.parametrize("opts", [dict(crossover=-1), dict(leaf=4), dict(leaf=16)])
def test_level_routes_and_leaf_sizes(torch_cuda, orc, opts):
    gamma, M, N = 1.4, 100, 333
    f, u0, phi = case(gamma, M, N, seed=5)
    (u,) = gpu_solve(torch_cuda, [(gamma, M, N)], [(f, u0, phi)], **opts)
    ref = orc.solve_cn(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    assert_parity(u, ref, gamma, M, N, f, u0, phi)


def test_multipass_levels_single_mode(torch_cuda, orc):
    # N > 8192: the largest levels take the multi-pass FFT route; one sine
    # mode keeps the oracle's check to a scalar recurrence
    gamma, M, N, j = 1.5, 64, 20000, 3
    x = np.arange(1, M + 1) / (M + 1)
    s = np.sin(j * np.pi * x)
    lam = 4.0 * (M + 1) ** 2 * math.sin(j * math.pi / (2 * (M + 1))) ** 2
    th = (np.arange(1, N + 1) - 0.5) / N
    g = 1 + th ** 2
    (u,) = gpu_solve(torch_cuda, [(gamma, M, N)], [(np.outer(g, s), 0.5 * s, -0.25 * s)])
    v = orc.mode_cn(gamma, 1.0, N, lam, g, 0.5, -0.25)
    assert relerr(u, np.outer(v, s)) <= TOL, relerr(u, np.outer(v, s))


def test_batch(torch_cuda, orc):
    probs = [(1.2, 64, 100), (1.7, 200, 64), (1.5, 1, 33), (1.9, 513, 40)]
    fields = [case(g, M, N, seed=k) for k, (g, M, N) in enumerate(probs)]
    us = gpu_solve(torch_cuda, probs, fields)
    for (g, M, N), (f, u0, phi), u in zip(probs, fields, us):
        ref = orc.solve_cn(g, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
        assert_parity(u, ref, g, M, N, f, u0, phi)


@pytest.mark.parametrize("M,N", [(37, 50), (256, 200), (2048, 33)])
def test_apply(torch_cuda, orc, M, N):
    gamma = 1.6
    rng = np.random.default_rng(M)
    U = rng.standard_normal((N, M))
    s = solver([(gamma, M, N)])
    y = s.apply([dev(torch_cuda, U)])[0].cpu().numpy()
    s.close()
    ref = orc.apply_cn(gamma, 1.0, 0.0, 1.0, M, N, U)
    assert relerr(y, ref) <= TOL, relerr(y, ref)


def test_adjoint_dot_identity(torch_cuda):
    """<A^-T g, f> = <g, A^-1 f> (zero initial data)."""
    gamma, M, N = 1.6, 300, 150
    rng = np.random.default_rng(8)
    f = rng.standard_normal((N, M))
    g = rng.standard_normal((N, M))
    s = solver([(gamma, M, N)])
    u = s.solve([dev(torch_cuda, f)])[0]
    lam = s.adjoint([dev(torch_cuda, g)], want_gamma=False)[0][0]
    torch_cuda.cuda.synchronize()
    lhs = float(np.sum(lam.cpu().numpy() * f))
    rhs = float(np.sum(g * u.cpu().numpy()))
    s.close()
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), np.linalg.norm(g) * np.linalg.norm(u.cpu().numpy())), (lhs, rhs)


@pytest.mark.parametrize("precond", [0, 1])
def test_gmres(torch_cuda, orc, precond):
    gamma, M, N = 1.3, 40, 48
    f, u0, phi = case(gamma, M, N, seed=2)
    s = solver([(gamma, M, N)])
    us, infos, _ = s.gmres([dev(torch_cuda, f)], [dev(torch_cuda, u0)], [dev(torch_cuda, phi)], restart=60,
                           max_iters=3000, rtol=1e-12, precond=precond)
    u = us[0].cpu().numpy()
    s.close()
    ref = orc.solve_cn(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    assert infos[0]["converged"] and relerr(u, ref) <= 1e-8, (infos[0], relerr(u, ref))


def test_rejected_settings(torch_cuda):
    from paper_1710_11593_amd import binding

    with pytest.raises(binding.FracsolveError, match="1 < gamma < 2"):
        solver([(0.5, 8, 8)])
    with pytest.raises(binding.FracsolveError, match="float64"):
        solver([(1.5, 8, 8)], precision="fp32", refine_steps=1)
    with pytest.raises(binding.FracsolveError, match="scan leaf"):
        solver([(1.5, 8, 8)], leaf_solver=1)


def test_full_size_c3_workload(torch_cuda, orc):
    """The c3 workload (diffusion-wave, gamma 1.5, M 2048, N 131072) in this
    variant, through single-mode reduction; where the float64 recurrence's
    own rounding exceeds 1e-11, against the extended-precision recurrence."""
    import bench
    from paper_1710_11593_amd import binding, workloads as wl

    inst = wl.c3(build=False)
    d = bench.device_inputs(inst, torch_cuda.device("cuda:0"))
    s = binding.Solver([dict(gamma=inst.gamma, M=inst.M, N=inst.N)], equation="diffusion_cn")
    u = s.solve([d["f"]], [d["u0"]], [d["phi"]])[0]
    torch_cuda.cuda.synchronize()
    s.close()
    err = bench.mode_error(inst, d, u, cn=True)
    print("c3 averaged spatial term: err vs oracle modes %.3e" % err, flush=True)
    if err <= TOL:
        return
    from tests import ext_reference
    from tests.test_gpu_parity import ext_mode_check

    e_gpu, e_orc, eta_gpu, eta_orc = ext_mode_check(torch_cuda, orc, inst, u, cn=True)
    ext_reference.assert_floor_parity(err, e_gpu, e_orc, eta_gpu, eta_orc, TOL)
