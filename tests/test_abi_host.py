"""Host-side checks of the C ABI and of the measurement plumbing (no GPU).

* every function include/fracsolve.h declares is exported by the built
  library and listed by the binding;
* argument errors are reported before any device work (E_ARG, with a
  message), so they are testable on a host without a GPU;
* the kernel names bench.py uses for the roofline match the dispatch tables
  of the FFT kernels, and the recorded-traffic lines of profiles/ parse.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fracsolve.h")
KFFT = os.path.join(ROOT, "paper_1710_11593_amd", "csrc", "k_fft.hip")

E_ARG, E_DEVICE = -1, -3


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(fracsolve_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1710_11593_amd import binding
    from paper_1710_11593_amd import build as hipbuild

    if not os.path.exists(binding.LIBPATH):
        hipbuild.build(force=False)
    return binding.lib()


def test_header_declares_the_binding_exports():
    from paper_1710_11593_amd import binding

    assert header_functions() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_function(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def create(lib, probs, opts=None):
    from paper_1710_11593_amd import binding

    arr = (binding.Problem * max(len(probs), 1))()
    for k, p in enumerate(probs):
        arr[k] = binding.Problem(*p)
    o = binding.Options(*(opts or (0, 0, 0, 0, 0, None)))
    h = ctypes.c_void_p()
    rc = lib.fracsolve_create(arr, len(probs), ctypes.byref(o), ctypes.byref(h))
    return rc, h, lib.fracsolve_last_error(None).decode()


GOOD = (0.5, 1.0, 0.0, 1.0, 64, 256)


@pytest.mark.parametrize("prob, pattern", [
    ((1.0, 1.0, 0.0, 1.0, 64, 256), "gamma"),
    ((2.0, 1.0, 0.0, 1.0, 64, 256), "gamma"),
    ((0.0, 1.0, 0.0, 1.0, 64, 256), "gamma"),
    ((0.5, 0.0, 0.0, 1.0, 64, 256), "T"),
    ((0.5, 1.0, 1.0, 1.0, 64, 256), "x1"),
    ((0.5, 1.0, 0.0, 1.0, 0, 256), "M"),
    ((0.5, 1.0, 0.0, 1.0, 4097, 256), "M"),
    ((0.5, 1.0, 0.0, 1.0, 64, 0), "N"),
    ((0.5, 1.0, 0.0, 1.0, 64, 131073), "N"),
])
def test_invalid_problem_is_rejected_before_device_work(lib, prob, pattern):
    rc, h, msg = create(lib, [GOOD, prob])
    assert rc == E_ARG and not h.value
    assert pattern in msg, msg


@pytest.mark.parametrize("opts, pattern", [
    ((3, 0, 0, 0, 0, None), "precision"),
    ((2, 1, 0, 0, 0, None), "not available"),   # split bf16 products are not built
    ((1, 9, 0, 0, 0, None), "refine_steps"),
    ((0, 0, 5, 0, 0, None), "leaf"),
    ((0, 0, 0, 0, 2, None), "leaf_solver"),
    ((0, 0, 0, 0, 0, None, 3), "equation"),
    ((0, 0, 0, 0, 0, None, 2), "1 < gamma < 2"),
    ((1, 1, 0, 0, 0, None, 1), "float64"),
    ((0, 0, 0, 0, 1, None, 1), "leaf_solver"),
    ((0, 0, 16, 0, 0, None, 1), "leaf"),
])
def test_invalid_options_are_rejected(lib, opts, pattern):
    rc, h, msg = create(lib, [GOOD], opts)
    assert rc == E_ARG and not h.value
    assert pattern in msg, msg


def test_empty_batch_and_null_handle(lib):
    rc, h, msg = create(lib, [])
    assert rc == E_ARG and "count" in msg
    lib.fracsolve_destroy(None)  # NULL-safe
    assert lib.fracsolve_solve(None, None, None, None, None) == E_ARG
    assert lib.fracsolve_set_check(None, 1) == E_ARG


def test_valid_problem_without_gpu_reports_no_device(lib):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, h, msg = create(lib, [GOOD])
    assert rc == E_DEVICE and not h.value, (rc, msg)


def dispatch_names():
    """n -> kernel text of the float64 update dispatch (FS_U2 / FS_U3 rows)."""
    text = open(KFFT).read()
    body = text[text.index("if constexpr (sizeof(T) == 8) {", text.index("if constexpr (MODE == MODE_UPDATE)")):]
    body = body[:body.index("} else {")]
    out = {}
    for m in re.finditer(r"FS_U2\((\d+), (\d+), (\d+)\)", body):
        n1, n2, cc = map(int, m.groups())
        out[n1 * n2] = "k_fft2u<double, %d, %d, %d, true>" % (n1, n2, cc)
    for m in re.finditer(r"FS_U3\((\d+), (\d+), (\d+), (\d+), (\d+)\)", body):
        n1, n2, n3, cc, nt = map(int, m.groups())
        out[n1 * n2 * n3] = "k_fft3u<double, %d, %d, %d, %d, %d, true>" % (n1, n2, n3, cc, nt)
    return out


def test_bench_kernel_names_match_the_dispatch():
    import bench

    assert bench.FFT64_NAMES == dispatch_names()


def test_recorded_traffic_lines_parse():
    """Every FFT level of the M = 4096 solve (s = 256 .. 32768) has one
    record; single-pass levels move about the algorithmic bytes, multi-pass
    levels (2 s > 8192) between 3 and 4.5 times them (the spectrum scratch
    is written once and read once in each direction)."""
    import bench

    path = os.path.join(ROOT, "profiles", "fft_level_traffic_M4096.md")
    lines = [l for l in open(path) if l.startswith("traffic:")]
    seen = set()
    for l in lines:
        m = re.match(r'traffic: s=(\d+) bytes_per_launch=(\d+) k_fft_sha=(\w{16})$', l.strip())
        assert m, l
        s, b = int(m.group(1)), int(m.group(2))
        alg = 24 * s * 4096
        if 2 * s in dispatch_names():
            assert 0.5 * alg <= b <= 1.5 * alg, l
        else:
            assert 3.0 * alg <= b <= 4.5 * alg, l
        assert bench.recorded_traffic(s, 4096) in (None, float(b))
        seen.add(s)
    assert seen == {256 << k for k in range(8)}


def ode_cg(lib, gamma, N, f=1, u=2, opts=None, hist=None, hist_cap=0):
    from paper_1710_11593_amd import binding

    o = binding.CgOptions(*opts) if opts else None
    info = binding.CgInfo()
    fn = lib.fracsolve_ode_cg
    fn.restype = ctypes.c_int
    rc = fn(ctypes.c_double(gamma), ctypes.c_int64(N), ctypes.c_void_p(f), ctypes.c_void_p(u),
            ctypes.byref(o) if o is not None else None, ctypes.byref(info), hist, ctypes.c_int32(hist_cap), None)
    return rc, lib.fracsolve_last_error(None).decode()


@pytest.mark.parametrize("gamma, N, kw, pattern", [
    (1.0, 64, {}, "gamma"),
    (0.0, 64, {}, "gamma"),
    (1.5, 64, {}, "gamma"),
    (0.5, 2, {}, "N must"),
    (0.5, 2 ** 22 + 2, {}, "N must"),
    (0.5, 64, {"f": 0}, "NULL"),
    (0.5, 64, {"u": 0}, "NULL"),
    (0.5, 64, {"opts": (-1, 1e-10, 0)}, "max_iters"),
    (0.5, 64, {"opts": (10, -1.0, 0)}, "rtol"),
    (0.5, 64, {"opts": (10, float("nan"), 0)}, "rtol"),
    (0.5, 64, {"opts": (10, 1e-10, 2)}, "use_guess"),
    (0.5, 64, {"hist_cap": 5}, "hist"),
])
def test_ode_cg_rejects_bad_arguments_before_device_work(lib, gamma, N, kw, pattern):
    # every check runs on the host before any device call, so the dummy
    # pointers are never touched
    rc, msg = ode_cg(lib, gamma, N, **kw)
    assert rc == E_ARG, (rc, msg)
    assert pattern in msg, msg


def test_ode_cg_valid_arguments_without_gpu_report_no_device(lib):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, msg = ode_cg(lib, 0.5, 2 ** 22 + 1)
    assert rc == E_DEVICE, (rc, msg)


@pytest.mark.parametrize("gamma, N, hist_cap, pattern", [
    (1.5, 1025, 0, "gamma"),
    (0.5, 2 ** 19 + 2, 0, "fixed workspace"),
    (0.5, 2 ** 22 + 1, 0, "fixed workspace"),
    (0.5, 1025, 65537, "fixed history"),
])
def test_ode_cg_noalloc_rejects_sizes_beyond_its_workspace(lib, gamma, N, hist_cap, pattern):
    # checked on the host before the fixed array's address is taken
    hist = (ctypes.c_double * max(hist_cap, 1))()
    fn = lib.fracsolve_ode_cg_noalloc
    fn.restype = ctypes.c_int
    rc = fn(ctypes.c_double(gamma), ctypes.c_int64(N), ctypes.c_void_p(1), ctypes.c_void_p(2), None, None,
            hist if hist_cap else None, ctypes.c_int32(hist_cap), None)
    msg = lib.fracsolve_last_error(None).decode()
    assert rc == E_ARG, (rc, msg)
    assert pattern in msg, msg


def test_recorded_full_run_parses():
    """The whole-run oracle time behind the cpu_baseline scaling is recorded
    for the c2 workload, with a ratio above the quadratic 64 (its later
    blocks run slower than a quadratic cost predicts) and is not applied to
    other workloads or sample sizes."""
    import bench

    rec = bench.recorded_full_run("c2", 4096, 65536, 0.3, 8192)
    assert rec and rec["threads"] >= 1
    assert 64.0 <= rec["total_s"] / rec["first_s"] <= 100.0
    assert bench.recorded_full_run("c2", 4096, 65536, 0.7, 8192) is None
    assert bench.recorded_full_run("c2", 4096, 65536, 0.3, 4096) is None
    assert bench.recorded_full_run("c3", 2048, 131072, 1.5, 8192) is None
