"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Floating-point bar: max-norm relative error <= 1e-11 for the float64 path
(the reading of the target agreement; rounding orders differ between the
recursive solve and time stepping), <= 1e-5 for the mixed forms after one
refinement step.  Sizes span several leaves and levels plus ragged tails.
"""
import math

import numpy as np
import pytest

from paper_1710_11593_amd import workloads as wl

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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def relerr(x, ref):
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def rand_case(gamma, M, N, seed=0):
    rng = np.random.default_rng(seed)
    x, t, _, _ = wl.grid(M, N)
    ts = wl.sample_times(gamma, N)
    f = np.outer(1 + ts ** 1.5, np.sin(np.pi * x)) + 0.3 * rng.standard_normal((N, M))
    u0 = np.sin(2 * np.pi * x) + 0.1 * rng.standard_normal(M)
    phi = np.cos(np.pi * x) if gamma > 1 else None
    return f, u0, phi


def gpu_weights(gamma, N):
    """The float64 weights a, rho, psi the library computes for (gamma, N)
    (the same for every width)."""
    from paper_1710_11593_amd import binding

    s = binding.Solver([dict(gamma=gamma, M=1, N=N)])
    w = s.weights(0)
    s.close()
    return w


def orc_weights(gamma, N):
    import oracle

    return oracle.weights(gamma, 1.0, N)


def assert_parity64(u, ref, gamma, M, N, f, u0, phi):
    """float64 bar: <= 1e-11 against the oracle.  Where the oracle's own
    float64 error exceeds that (the floor regime: its distance to an
    extended-precision solve of the same system), both results are checked
    against the extended solve (forward error <= 1e-8) and by their backward
    errors: the GPU's at most 8 ulp or twice the oracle's."""
    e = relerr(u, ref)
    if e <= TOL64:
        return
    from tests import ext_reference

    ext = np.asarray(ext_reference.solve(gamma, M, N, f, u0, phi), dtype=np.float64)
    e_gpu, e_orc = relerr(u, ext), relerr(ref, ext)
    eta_gpu = ext_reference.backward(gpu_weights(gamma, N), M, N, f, u, u0, phi)
    eta_orc = ext_reference.backward(orc_weights(gamma, N), M, N, f, ref, u0, phi)
    print("  floor: vs extended gpu %.2e oracle %.2e; backward error gpu %.2f oracle %.2f ulp"
          % (e_gpu, e_orc, eta_gpu / ext_reference.EPS, eta_orc / ext_reference.EPS), flush=True)
    ext_reference.assert_floor_parity(e, e_gpu, e_orc, eta_gpu, eta_orc, TOL64)


def gpu_solve(torch, gamma, M, N, f, u0=None, phi=None, **opts):
    from paper_1710_11593_amd import binding

    s = binding.Solver([dict(gamma=gamma, M=M, N=N)], **opts)
    u = s.solve([dev(torch, f)], [dev(torch, u0)] if u0 is not None else None,
                [dev(torch, phi)] if phi is not None else None)[0]
    torch.cuda.synchronize()
    out = u.cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("gamma", [0.1, 0.5, 0.9, 1.1, 1.5, 1.9])
def test_weights_vs_oracle(torch_cuda, orc, gamma):
    from paper_1710_11593_amd import binding

    N = 4096
    s = binding.Solver([dict(gamma=gamma, M=8, N=N)])
    w = s.weights(0)
    s.close()
    o = orc.weights(gamma, 1.0, N)
    eps = np.finfo(float).eps
    assert np.max(np.abs(w["b"] - o["b"]) / o["b"]) <= 4 * eps
    scale = o["coef"] * np.maximum(np.abs(o["b"]), np.abs(np.roll(o["b"], 2)))
    assert np.all(np.abs(w["a"] - o["a"]) <= 8 * eps * scale + 1e-300)
    for k in ("rho", "psi"):
        assert np.max(np.abs(w[k] - o[k])) <= 8 * eps * o["coef"]
    for k in ("da", "drho", "dpsi"):
        sc = np.max(np.abs(o[k])) + 1e-300
        assert np.max(np.abs(w[k] - o[k])) <= 1e-12 * sc, k
    # each a_m to a few ulp of itself against 40-digit decimal (the
    # diffusion-wave recurrence turns a relative weight error of 1e-16 into
    # about 1e-12 on the solution at N = 8192, so the weights must not lose
    # bits to cancellation)
    from tests import ext_reference

    a_dec, rho_dec, psi_dec = ext_reference.weights(gamma, N)
    rel = np.abs((np.asarray(w["a"], dtype=np.longdouble) - a_dec) / a_dec)
    assert float(np.max(rel)) <= 16 * eps, (int(np.argmax(rel)), float(np.max(rel)))
    for k, ref in (("rho", rho_dec), ("psi", psi_dec)):
        ref = np.asarray(ref, dtype=np.longdouble)
        nz = ref != 0
        if np.any(nz):
            assert float(np.max(np.abs((w[k][nz] - ref[nz]) / ref[nz]))) <= 16 * eps, k


@pytest.mark.parametrize("leaf_solver", [0, 1])
@pytest.mark.parametrize("crossover", [-1, 64, 1024])
@pytest.mark.parametrize("leaf", [4, 8, 16])
def test_c1_parity(torch_cuda, orc, crossover, leaf, leaf_solver):
    """c1 (diffusion, gamma=0.5, M=64, N=256), every level as FFT, default, or
    dense; both leaf solvers."""
    inst = wl.c1()
    ref = orc.solve(inst.gamma, 1.0, 0.0, 1.0, inst.M, inst.N, inst.f, u0=inst.u0)
    u = gpu_solve(torch_cuda, inst.gamma, inst.M, inst.N, inst.f, inst.u0, crossover=crossover, leaf=leaf,
                  leaf_solver=leaf_solver)
    assert relerr(u, ref) <= TOL64
    _, _, _, exact = wl.manufactured_source(inst.gamma, inst.M, inst.N)
    assert relerr(u, exact) < 1e-3  # discretisation error of the scheme, reported in the design doc


@pytest.mark.parametrize("gamma,M,N", [
    (0.3, 50, 200),      # ragged N, M not a multiple of the row blocking
    (0.7, 1, 37),        # single interior point
    (0.7, 2, 9),
    (1.3, 3, 1),         # a single time step
    (1.6, 129, 130),     # just above a power of two in both
    (0.45, 511, 300),
    (1.75, 1000, 257),
    (0.8, 2048, 96),
    (0.2, 4096, 40),     # largest M
    (1.2, 4095, 33),
])
@pytest.mark.parametrize("crossover,leaf_solver", [(-1, 0), (0, 0), (0, 1)])
def test_ragged_parity(torch_cuda, orc, gamma, M, N, crossover, leaf_solver):
    """Rough random sources, ragged sizes, both leaf solvers."""
    f, u0, phi = rand_case(gamma, M, N, seed=M + N)
    ref = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    u = gpu_solve(torch_cuda, gamma, M, N, f, u0, phi, crossover=crossover, leaf_solver=leaf_solver)
    assert_parity64(u, ref, gamma, M, N, f, u0, phi)


@pytest.mark.parametrize("gamma,M,N", [(0.3, 4096, 256), (0.7, 4096, 128), (1.5, 2048, 256), (0.6, 1024, 512)])
def test_smooth_workload_parity(torch_cuda, orc, gamma, M, N):
    """Workload-shaped input (manufactured source + seeded sine modes) at the
    configurations' M: float64 agreement <= 1e-11."""
    inst = wl.Instance(gamma, M, N, modes=[(j, a, p) for j, a, p in zip(
        range(1, 9), np.random.default_rng(2).standard_normal(8), np.random.default_rng(3).uniform(1, 3, 8))],
        manufactured=True)
    wl.fill(inst)
    ref = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, inst.f, u0=inst.u0, phi=inst.phi)
    for cross in (-1, 0):
        u = gpu_solve(torch_cuda, gamma, M, N, inst.f, inst.u0, inst.phi if gamma > 1 else None, crossover=cross)
        assert_parity64(u, ref, gamma, M, N, inst.f, inst.u0, inst.phi if gamma > 1 else None)


@pytest.mark.parametrize("gamma", [0.4, 1.4])
@pytest.mark.parametrize("crossover", [-1, 0])
def test_multipass_fft_level(torch_cuda, orc, gamma, crossover):
    """N = 20000 -> Np = 32768: levels with 2s = 16384, 32768 take the
    multi-pass FFT.  Sine-mode source with seeded random time profiles,
    against the exact discrete solution from the single-mode recurrences."""
    from paper_1710_11593_amd import binding

    rng = np.random.default_rng(7)
    inst = wl.Instance(gamma, 6, 20000, modes=[(j, float(a), float(p)) for j, a, p in zip(
        (1, 2, 5), rng.standard_normal(3), rng.uniform(1, 3, 3))], manufactured=True)
    f, u0, phi, ref = mode_reference(torch_cuda, orc, inst)
    s = binding.Solver([dict(gamma=gamma, M=inst.M, N=inst.N)], crossover=crossover)
    u = s.solve([f], [u0], [phi] if gamma > 1 else None)[0]
    torch_cuda.cuda.synchronize()
    s.close()
    err = float((u - ref).abs().max() / ref.abs().max())
    if err > TOL64:
        # float64 floor of the diffusion-wave recurrence: measure it
        from tests import ext_reference

        e_gpu, e_orc, eta_gpu, eta_orc = ext_mode_check(torch_cuda, orc, inst, u)
        ext_reference.assert_floor_parity(err, e_gpu, e_orc, eta_gpu, eta_orc, TOL64)


def test_multipass_levels_in_small_column_chunks(torch_cuda, orc, monkeypatch):
    """The multi-pass levels (2s = 16384, 32768 at N = 20000) of a width
    whose complex columns (500) split into ragged chunks of the smallest
    scratch (16 MiB: 64 and 32 columns per chunk): the same bits as one
    chunk per level, and the mode-reduction reference."""
    from paper_1710_11593_amd import binding

    rng = np.random.default_rng(11)
    inst = wl.Instance(0.4, 1000, 20000, modes=[(j, float(a), float(p)) for j, a, p in zip(
        (1, 3, 7), rng.standard_normal(3), rng.uniform(1, 3, 3))], manufactured=True)
    f, u0, phi, ref = mode_reference(torch_cuda, orc, inst)
    us = []
    for mb in ("4096", "16"):
        monkeypatch.setenv("FRACSOLVE_MP_SCRATCH_MB", mb)
        s = binding.Solver([dict(gamma=inst.gamma, M=inst.M, N=inst.N)], crossover=-1)
        us.append(s.solve([f], [u0])[0])
        torch_cuda.cuda.synchronize()
        s.close()
    assert torch_cuda.equal(us[0], us[1])
    err = float((us[1] - ref).abs().max() / ref.abs().max())
    assert err <= TOL64, err


@pytest.mark.parametrize("gamma,M,N", [(0.6, 33, 100), (1.5, 64, 128), (0.9, 300, 77)])
def test_apply_parity(torch_cuda, orc, gamma, M, N):
    from paper_1710_11593_amd import binding

    rng = np.random.default_rng(1)
    x = rng.standard_normal((N, M))
    ref = orc.apply(gamma, 1.0, 0.0, 1.0, M, N, x)
    for cross in (-1, 0):
        s = binding.Solver([dict(gamma=gamma, M=M, N=N)], crossover=cross)
        y = s.apply([dev(torch_cuda, x)])[0].cpu().numpy()
        s.close()
        assert relerr(y, ref) <= TOL64


@pytest.mark.parametrize("gamma,M,N", [(0.6, 40, 96), (1.4, 17, 50), (0.3, 128, 256), (0.7, 1000, 64), (1.3, 2048, 40)])
def test_adjoint_parity(torch_cuda, orc, gamma, M, N):
    from paper_1710_11593_amd import binding

    f, u0, phi = rand_case(gamma, M, N, seed=3)
    rng = np.random.default_rng(9)
    U = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    g = rng.standard_normal((N, M))
    lam_ref, dg_ref = orc.adjoint(gamma, 1.0, 0.0, 1.0, M, N, g, U, u0, phi)
    s = binding.Solver([dict(gamma=gamma, M=M, N=N)])
    lam, dg = s.adjoint([dev(torch_cuda, g)], [dev(torch_cuda, U)], [dev(torch_cuda, u0)],
                        [dev(torch_cuda, phi)] if phi is not None else None)
    lam = lam[0].cpu().numpy()
    s.close()
    e = relerr(lam, lam_ref)
    if e > TOL64:
        # the adjoint is the time-reversed solve of the same system with
        # right-hand side g: measure the oracle's own float64 floor there
        from tests import ext_reference

        ext = np.asarray(ext_reference.solve(gamma, M, N, g[::-1]), dtype=np.float64)[::-1]
        e_gpu, e_orc = relerr(lam, ext), relerr(lam_ref, ext)
        # backward errors of the time-reversed forward systems they solve
        eta_gpu = ext_reference.backward(gpu_weights(gamma, N), M, N, g[::-1], lam[::-1])
        eta_orc = ext_reference.backward(orc_weights(gamma, N), M, N, g[::-1], lam_ref[::-1])
        print("  floor: vs extended gpu %.2e oracle %.2e; backward error gpu %.2f oracle %.2f ulp"
              % (e_gpu, e_orc, eta_gpu / ext_reference.EPS, eta_orc / ext_reference.EPS), flush=True)
        ext_reference.assert_floor_parity(e, e_gpu, e_orc, eta_gpu, eta_orc, TOL64)
    assert abs(dg[0] - dg_ref) <= 1e-10 * abs(dg_ref)


@pytest.mark.parametrize("precision", ["fp32"])
@pytest.mark.parametrize("gamma,M,N", [(0.5, 64, 256), (1.5, 128, 512), (0.3, 1000, 300)])
def test_mixed_precision_refined(torch_cuda, orc, precision, gamma, M, N):
    # crossover 16: the levels from s = 32 up are float32 FFT products (the
    # tuned plan keeps every level of sizes this small dense, in float64)
    f, u0, phi = rand_case(gamma, M, N, seed=5)
    ref = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    u0r = gpu_solve(torch_cuda, gamma, M, N, f, u0, phi, precision=precision, refine_steps=0, crossover=16)
    u1 = gpu_solve(torch_cuda, gamma, M, N, f, u0, phi, precision=precision, refine_steps=1, crossover=16)
    e0, e1 = relerr(u0r, ref), relerr(u1, ref)
    assert e1 <= 1e-5, (e0, e1)
    assert e1 <= e0


@pytest.mark.parametrize("gamma", [0.02, 0.98, 1.02, 1.98])
def test_gamma_near_the_regime_ends(torch_cuda, orc, gamma):
    """Orders close to 0, 1 and 2 (weights that nearly vanish or nearly
    cancel), several levels and a ragged tail, against the oracle."""
    M, N = 100, 600
    f, u0, phi = rand_case(gamma, M, N, seed=7)
    u = gpu_solve(torch_cuda, gamma, M, N, f, u0, phi)
    ref = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    assert_parity64(u, ref, gamma, M, N, f, u0, phi)


def test_batched_parity(torch_cuda, orc):
    from paper_1710_11593_amd import binding

    cases = [(0.3, 64, 256), (1.2, 200, 100), (0.8, 1500, 64), (1.9, 7, 1000), (0.5, 4096, 16)]
    data = [rand_case(g, M, N, seed=i) for i, (g, M, N) in enumerate(cases)]
    s = binding.Solver([dict(gamma=g, M=M, N=N) for g, M, N in cases])
    us = s.solve([dev(torch_cuda, d[0]) for d in data], [dev(torch_cuda, d[1]) for d in data],
                 [dev(torch_cuda, d[2]) if d[2] is not None else None for d in data])
    torch_cuda.cuda.synchronize()
    for (g, M, N), d, u in zip(cases, data, us):
        ref = orc.solve(g, 1.0, 0.0, 1.0, M, N, d[0], u0=d[1], phi=d[2])
        assert_parity64(u.cpu().numpy(), ref, g, M, N, d[0], d[1], d[2])
    s.close()


def test_batched_parity_narrow(torch_cuda, orc):
    """A batch whose widest instance has M <= 2048 (the batch leaf
    configuration differs from the single-instance one there)."""
    from paper_1710_11593_amd import binding

    cases = [(0.3, 1500, 300), (1.4, 77, 500), (0.6, 600, 200), (1.8, 2048, 130)]
    data = [rand_case(g, M, N, seed=10 + i) for i, (g, M, N) in enumerate(cases)]
    s = binding.Solver([dict(gamma=g, M=M, N=N) for g, M, N in cases])
    us = s.solve([dev(torch_cuda, d[0]) for d in data], [dev(torch_cuda, d[1]) for d in data],
                 [dev(torch_cuda, d[2]) if d[2] is not None else None for d in data])
    torch_cuda.cuda.synchronize()
    for (g, M, N), d, u in zip(cases, data, us):
        ref = orc.solve(g, 1.0, 0.0, 1.0, M, N, d[0], u0=d[1], phi=d[2])
        assert_parity64(u.cpu().numpy(), ref, g, M, N, d[0], d[1], d[2])
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_widths_multipass(torch_cuda, orc, precision):
    """A batch of instances of four widths (every instance runs the leaf
    kernel of the widest one, so each step is one leaf launch; rows are
    accessed per element or in 16-byte units per task), with multi-pass FFT
    levels (Np > 8192) in several instances.  Each instance is checked
    against the single-mode oracle reference within the bar of its form, and
    against its own single-instance solve (a different leaf configuration,
    so a different rounding order)."""
    from paper_1710_11593_amd import binding

    specs = [(0.4, 100, 20000), (1.3, 401, 12000), (0.7, 1000, 9000), (1.6, 3000, 16384)]
    insts = []
    for k, (g, M, N) in enumerate(specs):
        rng = np.random.default_rng(40 + k)
        amps, pows = wl.random_modes(rng, 3)
        insts.append(wl.Instance(g, M, N, modes=[(j, float(a), float(p)) for j, a, p in zip((2, 5, 9), amps, pows)],
                                 manufactured=True))
    data = [mode_reference(torch_cuda, orc, inst) for inst in insts]
    refine = 1 if precision == "fp32" else 0
    bar = 1e-5 if precision == "fp32" else 1e-9
    probs = [dict(gamma=i.gamma, M=i.M, N=i.N) for i in insts]
    s = binding.Solver(probs, precision=precision, refine_steps=refine)
    us = s.solve([d[0] for d in data], [d[1] for d in data], [d[2] if i.gamma > 1 else None for d, i in zip(data, insts)])
    torch_cuda.cuda.synchronize()
    s.close()
    for inst, d, u in zip(insts, data, us):
        err = float((u - d[3]).abs().max() / d[3].abs().max())
        assert err <= bar, (inst.gamma, inst.M, inst.N, err)
        one = binding.Solver([dict(gamma=inst.gamma, M=inst.M, N=inst.N)], precision=precision, refine_steps=refine)
        u1 = one.solve([d[0]], [d[1]], [d[2]] if inst.gamma > 1 else None)[0]
        torch_cuda.cuda.synchronize()
        one.close()
        diff = float((u - u1).abs().max() / u1.abs().max())
        assert diff <= bar, (inst.gamma, inst.M, inst.N, diff)


def test_graph_replay_matches_eager(torch_cuda, orc, monkeypatch):
    """Recorded launch sequences (FRACSOLVE_GRAPH=1) replayed several times,
    with eager work and synchronisations in between, give the eager result."""
    from paper_1710_11593_amd import binding

    gamma, M, N = 0.4, 200, 300
    cases = [rand_case(gamma, M, N, seed=s) for s in range(3)]
    eager = [gpu_solve(torch_cuda, gamma, M, N, f, u0) for f, u0, _ in cases]
    monkeypatch.setenv("FRACSOLVE_GRAPH", "1")
    s = binding.Solver([dict(gamma=gamma, M=M, N=N)])
    for rep in range(3):
        for (f, u0, _), ref in zip(cases, eager):
            u = s.solve([dev(torch_cuda, f)], [dev(torch_cuda, u0)])[0]
            torch_cuda.cuda.synchronize()
            _ = torch_cuda.ones(1000, device="cuda").sum().item()  # eager work in between
            assert np.array_equal(u.cpu().numpy(), ref), rep
    s.close()


def mode_reference(torch, orc, inst):
    """Exact discrete solution of a sum-of-sine-modes instance through the
    single-mode scalar recurrences (P5), assembled on the GPU."""
    import math
    from concurrent.futures import ThreadPoolExecutor

    series = wl.modal_time_series(inst)
    js = sorted(series)
    x, _, h, _ = wl.grid(inst.M, inst.N)
    S = np.stack([np.sin(j * math.pi * x) for j in js])
    lam = [4.0 / h ** 2 * math.sin(j * math.pi * h / 2) ** 2 for j in js]
    with ThreadPoolExecutor(max_workers=len(js)) as ex:
        vs = list(ex.map(lambda k: orc.mode(inst.gamma, inst.T, inst.N, lam[k], series[js[k]][0],
                                            series[js[k]][1], series[js[k]][2]), range(len(js))))
    G = np.stack([series[j][0] for j in js], axis=1)
    Sd = torch.from_numpy(S).cuda()
    f = torch.from_numpy(G).cuda() @ Sd
    u0 = torch.from_numpy(np.array([series[j][1] for j in js]) @ S).cuda()
    phi = torch.from_numpy(np.array([series[j][2] for j in js]) @ S).cuda()
    ref = torch.from_numpy(np.stack(vs, axis=1)).cuda() @ Sd
    return f, u0, phi, ref


def ext_mode_check(torch, orc, inst, u, cn=False):
    """Floor-regime measures of a sum-of-sine-modes instance: (GPU forward
    error, float64 oracle recurrence forward error), both against the
    extended-precision recurrence, and (GPU backward error, oracle backward
    error), each for the system its own float64 weights define (the GPU's
    modal coefficients by projection of its field)."""
    import math

    from tests import ext_reference

    series = wl.modal_time_series(inst)
    x, _, h, _ = wl.grid(inst.M, inst.N)
    js = sorted(series)
    uext, uorc, v64s = None, None, {}
    for j in js:
        g, v0, ph = series[j]
        lam = 4.0 / h ** 2 * math.sin(j * math.pi * h / 2) ** 2
        vx = ext_reference.mode(inst.gamma, inst.T, inst.N, lam, g, v0, ph, cn=cn)
        v64 = (orc.mode_cn if cn else orc.mode)(inst.gamma, inst.T, inst.N, lam, g, v0, ph)
        v64s[j] = v64
        sj = torch.from_numpy(np.sin(j * math.pi * x)).cuda()[None, :]
        term = torch.from_numpy(vx).cuda()[:, None] * sj
        tor = torch.from_numpy(v64).cuda()[:, None] * sj
        uext = term if uext is None else uext + term
        uorc = tor if uorc is None else uorc + tor
    nrm = float(uext.abs().max())
    e_gpu = float((u - uext).abs().max()) / nrm
    e_orc = float((uorc - uext).abs().max()) / nrm
    vg = dict(zip(js, ext_reference.modal_coefficients(u, js)))
    eta_gpu = ext_reference.modal_backward(gpu_weights(inst.gamma, inst.N), inst.M, inst.N, series, vg, cn=cn)
    eta_orc = ext_reference.modal_backward(orc.weights(inst.gamma, inst.T, inst.N), inst.M, inst.N, series, v64s,
                                           cn=cn)
    print("  floor: vs extended gpu %.2e oracle %.2e; backward error gpu %.2f oracle %.2f ulp"
          % (e_gpu, e_orc, eta_gpu / ext_reference.EPS, eta_orc / ext_reference.EPS), flush=True)
    return e_gpu, e_orc, eta_gpu, eta_orc


@pytest.mark.parametrize("which", ["c2-0.3", "c2-0.7", "c3"])
def test_full_size_mode_reduction(torch_cuda, orc, which):
    """Full configuration sizes (M=4096, N=2^16; M=2048, N=2^17) in the bench's
    launch configuration, against the discrete solution assembled from the
    oracle's single-mode recurrences.  For the diffusion-wave case (c3) the
    float64 recurrence itself carries a rounding floor well above 1e-11 at
    N = 2^17 (the history sum cancels several times the result at every
    step); there the floor regime's checks apply (extended-precision
    recurrence, backward errors)."""
    from paper_1710_11593_amd import binding
    from tests import ext_reference

    if which.startswith("c2"):
        g = float(which.split("-")[1])
        inst = wl.c2(gamma=g, seed=3 if g == 0.7 else 2, build=False)  # the recipe's seeds
    else:
        inst = wl.c3(build=False)
    f, u0, phi, ref = mode_reference(torch_cuda, orc, inst)
    s = binding.Solver([dict(gamma=inst.gamma, M=inst.M, N=inst.N)])
    u = s.solve([f], [u0], [phi] if inst.gamma > 1 else None)[0]
    torch_cuda.cuda.synchronize()
    s.close()
    err = float((u - ref).abs().max() / ref.abs().max())
    print("%s: max-norm relative error vs the float64 single-mode reference %.3e" % (which, err))
    if which.startswith("c2") or err <= TOL64:
        assert err <= TOL64
        return
    # c3: the float64 floor of the diffusion-wave recurrence at N = 2^17
    e_gpu, e_orc, eta_gpu, eta_orc = ext_mode_check(torch_cuda, orc, inst, u)
    print("c3: GPU vs extended %.3e, float64 oracle recurrence vs extended %.3e" % (e_gpu, e_orc))
    ext_reference.assert_floor_parity(err, e_gpu, e_orc, eta_gpu, eta_orc, TOL64)


@pytest.mark.parametrize("gamma,M,N", [(0.35, 5, 2048), (1.45, 33, 1500), (0.8, 1000, 1100), (1.7, 2048, 300)])
def test_dense_levels_on_the_matrix_cores(torch_cuda, orc, gamma, M, N):
    """Crossover 512: the dense level products of half-size 128..512 run on
    the float64 matrix cores (16x16x4 MFMA tiles over 16-column slabs), the
    smaller ones on the vector units; ragged widths (slabs past M) and row
    counts (the last level's Y block cut at N)."""
    f, u0, phi = rand_case(gamma, M, N, seed=N)
    ref = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0, phi=phi)
    u = gpu_solve(torch_cuda, gamma, M, N, f, u0, phi, crossover=512)
    assert_parity64(u, ref, gamma, M, N, f, u0, phi)


def test_dense_mfma_apply_and_batch(torch_cuda, orc):
    """The matrix-core dense products in the operator apply and in a batch
    of uneven instances (one launch over every task of a level)."""
    from paper_1710_11593_amd import binding

    rng = np.random.default_rng(11)
    M, N = 70, 1300
    x = rng.standard_normal((N, M))
    s = binding.Solver([dict(gamma=0.55, M=M, N=N)], crossover=512)
    y = s.apply([dev(torch_cuda, x)])[0].cpu().numpy()
    s.close()
    assert relerr(y, orc.apply(0.55, 1.0, 0.0, 1.0, M, N, x)) <= TOL64
    cases = [(0.3, 17, 900), (1.2, 300, 1200), (0.6, 64, 513)]
    data = [rand_case(g, Mi, Ni, seed=20 + i) for i, (g, Mi, Ni) in enumerate(cases)]
    s = binding.Solver([dict(gamma=g, M=Mi, N=Ni) for g, Mi, Ni in cases], crossover=512)
    us = s.solve([dev(torch_cuda, d[0]) for d in data], [dev(torch_cuda, d[1]) for d in data],
                 [dev(torch_cuda, d[2]) if d[2] is not None else None for d in data])
    torch_cuda.cuda.synchronize()
    for (g, Mi, Ni), d, u in zip(cases, data, us):
        ref = orc.solve(g, 1.0, 0.0, 1.0, Mi, Ni, d[0], u0=d[1], phi=d[2])
        assert_parity64(u.cpu().numpy(), ref, g, Mi, Ni, d[0], d[1], d[2])
    s.close()


def test_output_check_reports_non_finite_values(torch_cuda, orc):
    """fracsolve_set_check: a finite solve passes unchanged (and equals the
    oracle); a NaN in one source row makes every later row non-finite, which
    the scan reports as E_NUMERIC naming the field and instance; apply and
    adjoint are checked the same way; off again, the same call returns OK."""
    from paper_1710_11593_amd import binding

    gamma, M, N = 0.6, 40, 96
    f, u0, _ = rand_case(gamma, M, N, seed=5)
    ref = orc.solve(gamma, 1.0, 0.0, 1.0, M, N, f, u0=u0)
    s = binding.Solver([dict(gamma=gamma, M=M, N=N)])
    s.set_check(True)
    u = s.solve([dev(torch_cuda, f)], [dev(torch_cuda, u0)])[0]
    assert relerr(u.cpu().numpy(), ref) <= TOL64
    bad = f.copy()
    bad[N // 2, M // 3] = np.nan
    with pytest.raises(binding.FracsolveError, match=r"E_NUMERIC.*u\[0\] holds \d+ non-finite"):
        s.solve([dev(torch_cuda, bad)], [dev(torch_cuda, u0)])
    x = np.ones((N, M))
    x[3, 4] = np.inf
    with pytest.raises(binding.FracsolveError, match=r"E_NUMERIC.*y\[0\]"):
        s.apply([dev(torch_cuda, x)])
    with pytest.raises(binding.FracsolveError, match=r"E_NUMERIC.*dL_df\[0\]"):
        s.adjoint([dev(torch_cuda, bad)], want_gamma=False)
    with pytest.raises(binding.FracsolveError, match=r"E_NUMERIC.*dL_dgamma\[0\] is not finite"):
        s.adjoint([dev(torch_cuda, bad)], [u], [dev(torch_cuda, u0)], None)
    s.set_check(False)
    s.solve([dev(torch_cuda, bad)], [dev(torch_cuda, u0)])
    s.close()
