"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, the ctypes structures match the C layout, and host-side argument
validation rejects bad inputs before any device call."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2107_00243_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpmll.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libgpmll.so is not built (run python -m paper_2107_00243_amd.build)")
    return B.load()


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(gp_\w+)\s*\(", src, re.M)))


def test_header_declares_the_bound_functions():
    assert declared_functions() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for name in declared_functions():
        assert name in syms, name
        assert hasattr(lib, name)


def test_struct_layouts_match_the_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#define __HIP_PLATFORM_AMD__ 1
#include <stdio.h>
#include <stddef.h>
#include "gpmll.h"
#define P(T, F) printf(#T "." #F " %zu\n", offsetof(T, F))
int main(void) {
  printf("gp_problem %zu\n", sizeof(gp_problem));
  printf("gp_options %zu\n", sizeof(gp_options));
  printf("gp_stats %zu\n", sizeof(gp_stats));
  printf("gp_precond_view %zu\n", sizeof(gp_precond_view));
  printf("gp_batch %zu\n", sizeof(gp_batch));
  printf("gp_batch_stats %zu\n", sizeof(gp_batch_stats));
  P(gp_batch, offsets_host); P(gp_batch, batch); P(gp_batch, ard);
  P(gp_batch_stats, flags_any); P(gp_batch_stats, iters_host); P(gp_batch_stats, rank_host);
  P(gp_problem, n); P(gp_problem, d); P(gp_problem, ard); P(gp_problem, kernel_shape);
  P(gp_options, cg_tol); P(gp_options, seed); P(gp_options, precond_grad); P(gp_options, sync_every);
  P(gp_options, probe_mode);
  P(gp_stats, logdet_precond); P(gp_stats, logdet_estimate); P(gp_stats, col_iters_host); P(gp_stats, pivots_host);
  P(gp_precond_view, n); P(gp_precond_view, rank);
  return 0;
}
''')
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include", str(prog), "-o",
                        str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], stdout=subprocess.PIPE,
                                                         text=True).stdout.splitlines())
    types = {"gp_problem": B.gp_problem, "gp_options": B.gp_options, "gp_stats": B.gp_stats,
             "gp_precond_view": B.gp_precond_view, "gp_batch": B.gp_batch, "gp_batch_stats": B.gp_batch_stats}
    for key, val in got.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(types[t], f).offset == int(val), key
        else:
            assert ctypes.sizeof(types[key]) == int(val), key


def test_a_plain_c_program_links_and_calls_the_library(tmp_path, lib):
    # the boundary needs nothing but the header and the shared library: a C program
    # linked against them sizes the workspace of the n = 100,000 bench shape and gets
    # the argument errors back, without a GPU (no call here reaches the device)
    prog = tmp_path / "consumer.c"
    prog.write_text(r"""
#define __HIP_PLATFORM_AMD__ 1
#include <stdio.h>
#include "gpmll.h"
int main(void) {
  gp_problem prob = {(const double*)0x1000, (const double*)0x2000, 100000, 16, GP_KERNEL_RBF, 1, 0.0};
  gp_options opt = {GP_PREC_BF16X3, 64, 200, 1e-6, 1, 0, 1, 0};
  size_t bytes = 0;
  int st = gp_workspace_size(&prob, &opt, 100, &bytes);
  printf("size %d %zu\n", st, bytes);
  prob.d = GP_MAX_D + 1;
  printf("bad_d %d\n", gp_workspace_size(&prob, &opt, 100, &bytes));
  prob.d = 16;
  double theta[18];
  for (int j = 0; j < 18; ++j) theta[j] = 1.0;
  printf("null_ws %d\n", gp_mll_grad(&prob, theta, &opt, 100, NULL, NULL, 0, NULL, NULL, NULL, NULL));
  printf("msg %s\n", gp_strerror(GP_EINVAL));
  return 0;
}
""")
    exe = tmp_path / "consumer"
    libdir = os.path.dirname(B.LIB_PATH)
    r = subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include", str(prog),
                        "-o", str(exe), "-L", libdir, "-l:" + os.path.basename(B.LIB_PATH),
                        "-Wl,-rpath," + libdir, "-L/opt/rocm/lib", "-lamdhip64"],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    out = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=60)
    assert out.returncode == 0, out.stdout
    got = dict(l.split(" ", 1) for l in out.stdout.splitlines())
    st, size = got["size"].split()
    prob = B.gp_problem(0x1000, 0x2000, 100000, 16, 0, 1)
    opt = B.make_options("bf16x3", 64, 200, 1e-6, 1, 0, 1)
    assert int(st) == 0 and int(size) == B.gp_workspace_size(prob, opt, 100)
    assert int(got["bad_d"]) == B.GP_EINVAL
    assert int(got["null_ws"]) == B.GP_EINVAL
    assert got["msg"].strip()


def _fake_problem(n=100, d=3, kernel=0, ard=1):
    return B.gp_problem(0x1000, 0x2000, n, d, kernel, ard)


def test_workspace_size_is_positive_and_grows(lib):
    o = B.make_options("bf16x3", 64, 200)
    s1 = B.gp_workspace_size(_fake_problem(1000, 16), o, 10)
    s2 = B.gp_workspace_size(_fake_problem(2000, 16), o, 10)
    assert 0 < s1 < s2


@pytest.mark.parametrize("mutate", [
    lambda p, o: setattr(p, "n", 0),
    lambda p, o: setattr(p, "d", 0),
    lambda p, o: setattr(p, "d", 33),
    lambda p, o: setattr(p, "kernel", 4),
    lambda p, o: setattr(p, "kernel", 3),              # rational quadratic without a shape
    lambda p, o: (setattr(p, "kernel", 3), setattr(p, "kernel_shape", float("nan"))),
    lambda p, o: setattr(p, "ard", 2),
    lambda p, o: setattr(o, "num_probes", 0),
    lambda p, o: setattr(o, "num_probes", 256),
    lambda p, o: setattr(o, "max_iters", 0),
    lambda p, o: setattr(o, "cg_tol", -1.0),
    lambda p, o: setattr(o, "cg_tol", float("nan")),
    lambda p, o: setattr(o, "precision", 4),
    lambda p, o: setattr(o, "precond_grad", 2),
    lambda p, o: setattr(o, "sync_every", -1),
    lambda p, o: setattr(o, "probe_mode", 2),
])
def test_invalid_shapes_and_options_are_rejected(lib, mutate):
    p, o = _fake_problem(), B.make_options("fp64", 4, 10)
    mutate(p, o)
    out = ctypes.c_size_t(0)
    r1 = lib.gp_workspace_size(ctypes.byref(p), ctypes.byref(o), 2, ctypes.byref(out))
    theta = np.array([0.5, 0.5, 0.5, 1.0, 0.1])
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    r2 = lib.gp_mll_eval(ctypes.byref(p), tp, ctypes.byref(o), 2, None, ctypes.c_void_p(0x10000), 1 << 30, None,
                         ctypes.c_void_p(0x3000), None)
    assert r1 == B.GP_EINVAL or r2 == B.GP_EINVAL
    assert r2 == B.GP_EINVAL


@pytest.mark.parametrize("bad", [0.0, -1.0, float("nan"), float("inf")])
@pytest.mark.parametrize("pos", [0, 3, 4])
def test_nonpositive_or_nan_theta_is_rejected(lib, bad, pos):
    p, o = _fake_problem(), B.make_options("fp64", 4, 10)
    theta = np.array([0.5, 0.5, 0.5, 1.0, 0.1])
    theta[pos] = bad
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    logp = ctypes.c_void_p(0x3000)
    assert lib.gp_mll_eval(ctypes.byref(p), tp, ctypes.byref(o), 2, None, ctypes.c_void_p(0x10000), 1 << 30, None,
                           logp, None) == B.GP_EINVAL
    assert lib.gp_mll_grad(ctypes.byref(p), tp, ctypes.byref(o), 2, None, ctypes.c_void_p(0x10000), 1 << 30, None,
                           logp, ctypes.c_void_p(0x4000), None) == B.GP_EINVAL
    h = ctypes.c_void_p()
    assert lib.gp_precond_build(ctypes.byref(p), tp, 2, ctypes.c_void_p(0x10000), 1 << 30, None,
                                ctypes.byref(h)) == B.GP_EINVAL


def test_null_pointers_and_rank_bounds_are_rejected(lib):
    o = B.make_options("fp64", 4, 10)
    theta = np.array([0.5, 0.5, 0.5, 1.0, 0.1])
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ws = ctypes.c_void_p(0x10000)
    p = _fake_problem()
    p_nox = B.gp_problem(0, 0x2000, 100, 3, 0, 1)
    for prob, rank, logp in ((p_nox, 2, 0x3000), (p, -1, 0x3000), (p, 101, 0x3000), (p, 2, 0)):
        assert lib.gp_mll_eval(ctypes.byref(prob), tp, ctypes.byref(o), rank, None, ws, 1 << 30, None,
                               ctypes.c_void_p(logp), None) == B.GP_EINVAL
    assert lib.gp_mll_grad(ctypes.byref(p), tp, ctypes.byref(o), 2, None, ws, 1 << 30, None,
                           ctypes.c_void_p(0x3000), None, None) == B.GP_EINVAL
    assert lib.gp_workspace_size(ctypes.byref(p), ctypes.byref(o), 2, None) == B.GP_EINVAL
    assert lib.gp_khat_matvec(ctypes.byref(p), tp, 0, None, 4, ctypes.c_void_p(0x5000), ws, 1 << 30, None) == B.GP_EINVAL
    assert lib.gp_khat_matvec(ctypes.byref(p), tp, 0, ctypes.c_void_p(0x5000), 0, ctypes.c_void_p(0x5000), ws,
                              1 << 30, None) == B.GP_EINVAL


def test_rff_build_rejects_odd_or_small_rank_and_null_frequencies(lib):
    theta = np.array([0.5, 0.5, 0.5, 1.0, 0.1])
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p = _fake_problem()
    ws = ctypes.c_void_p(0x10000)
    h = ctypes.c_void_p()
    for rank, freq in ((3, 0x6000), (0, 0x6000), (4, 0), (102, 0x6000)):
        assert lib.gp_precond_build_rff(ctypes.byref(p), tp, rank, ctypes.c_void_p(freq), ws, 1 << 30, None,
                                        ctypes.byref(h)) == B.GP_EINVAL
    assert lib.gp_precond_build_rff(ctypes.byref(p), tp, 4, ctypes.c_void_p(0x6000), ws, 1 << 30, None,
                                    None) == B.GP_EINVAL


def test_nystrom_build_rejects_bad_landmarks_before_any_device_call(lib):
    theta = np.array([0.5, 0.5, 0.5, 1.0, 0.1])
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p = _fake_problem()
    ws = ctypes.c_void_p(0x10000)
    h = ctypes.c_void_p()
    for lm in ([1, 2, 2, 3], [1, 2, 3, 100], [-1, 2, 3, 4]):
        a = np.array(lm, dtype=np.int32)
        assert lib.gp_precond_build_nystrom(ctypes.byref(p), tp, 4, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            ws, 1 << 30, None, ctypes.byref(h)) == B.GP_EINVAL
    assert lib.gp_precond_build_nystrom(ctypes.byref(p), tp, 4, None, ws, 1 << 30, None,
                                        ctypes.byref(h)) == B.GP_EINVAL


def test_qff_build_rejects_bad_node_counts_and_kernels(lib):
    theta = np.array([0.5, 0.5, 0.5, 1.0, 0.1])
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ws = ctypes.c_void_p(0x10000)
    h = ctypes.c_void_p()
    p = _fake_problem(n=10000, d=3)
    for q in (3, 0, 66, 12):   # odd, too small, above 64, 12^3 > GP_MAX_RANK
        assert lib.gp_precond_build_qff(ctypes.byref(p), tp, q, ws, 1 << 30, None, ctypes.byref(h)) == B.GP_EINVAL
    p_small = _fake_problem(n=50, d=3)   # 4^3 = 64 > n
    assert lib.gp_precond_build_qff(ctypes.byref(p_small), tp, 4, ws, 1 << 30, None, ctypes.byref(h)) == B.GP_EINVAL
    p_mat = _fake_problem(n=10000, d=3, kernel=1)
    assert lib.gp_precond_build_qff(ctypes.byref(p_mat), tp, 4, ws, 1 << 30, None,
                                    ctypes.byref(h)) == B.GP_EUNSUPPORTED


def test_predict_rejects_null_outputs_and_empty_test_sets(lib):
    theta = np.array([0.5, 0.5, 0.5, 1.0, 0.1])
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    o = B.make_options("fp64", 4, 10)
    p = _fake_problem()
    ws = ctypes.c_void_p(0x10000)
    xs, mean = ctypes.c_void_p(0x7000), ctypes.c_void_p(0x8000)
    for xs_, n_, m_ in ((None, 5, mean), (xs, 0, mean), (xs, 5, None)):
        assert lib.gp_predict(ctypes.byref(p), tp, ctypes.byref(o), 2, None, xs_, n_, ws, 1 << 30, None, m_,
                              None) == B.GP_EINVAL


def test_batch_reports_the_rational_quadratic_kernel_unsupported(lib):
    o = B.make_options("fp64", 4, 10)
    offs = (ctypes.c_int64 * 3)(0, 100, 250)
    b = B.gp_batch(0x1000, 0x2000, offs, 2, 3, 3, 1)
    out = ctypes.c_size_t(0)
    assert lib.gp_batch_workspace_size(ctypes.byref(b), ctypes.byref(o), 2, ctypes.byref(out)) == B.GP_EUNSUPPORTED


def test_batch_reports_square_root_probes_unsupported(lib):
    o = B.make_options("fp64", 4, 10, probe_mode=1)
    offs = (ctypes.c_int64 * 3)(0, 100, 250)
    b = B.gp_batch(0x1000, 0x2000, offs, 2, 3, 0, 1)
    out = ctypes.c_size_t(0)
    assert lib.gp_batch_workspace_size(ctypes.byref(b), ctypes.byref(o), 2, ctypes.byref(out)) == B.GP_EUNSUPPORTED


def test_square_root_probes_need_more_workspace(lib):
    p = _fake_problem(n=5000, d=3)
    s0 = B.gp_workspace_size(p, B.make_options("fp64", 8, 50), 200)
    s1 = B.gp_workspace_size(p, B.make_options("fp64", 8, 50, probe_mode=1), 200)
    assert s1 >= s0 + 6 * 200 * 200 * 8 - 256   # the empty slot of mode 0 still takes one 256-byte unit


def test_strerror_covers_every_status(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert B.gp_strerror(code) and B.gp_strerror(code) != "unknown status"
    assert B.gp_strerror(-99) == "unknown status"


def test_precond_free_accepts_null(lib):
    lib.gp_precond_free(None)


# ---------------------------------------------------------------- batched entry points

def _fake_batch(sizes=(10, 20, 5), d=3, kernel=0, ard=1):
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    b = B.gp_batch(0x1000, 0x2000, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(sizes), d, kernel, ard)
    return b, offs


def test_batch_workspace_size_grows_with_the_problems(lib):
    o = B.make_options("fp32", 16, 200)
    b1, k1 = _fake_batch((500, 800))
    b2, k2 = _fake_batch((500, 800, 3000))
    s1, s2 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.gp_batch_workspace_size(ctypes.byref(b1), ctypes.byref(o), 20, ctypes.byref(s1)) == B.GP_OK
    assert lib.gp_batch_workspace_size(ctypes.byref(b2), ctypes.byref(o), 20, ctypes.byref(s2)) == B.GP_OK
    assert 0 < s1.value < s2.value


@pytest.mark.parametrize("case", ["zero_size", "bad_first", "decreasing", "batch0", "d0", "d33", "kernel", "ard",
                                  "rank_neg"])
def test_batch_rejects_bad_shapes(lib, case):
    sizes = (10, 20, 5)
    b, offs = _fake_batch(sizes)
    o = B.make_options("fp64", 4, 10)
    rank = 2
    if case == "zero_size":
        offs[2] = offs[1]
    elif case == "bad_first":
        offs[0] = 1
    elif case == "decreasing":
        offs[2] = offs[1] - 1
    elif case == "batch0":
        b.batch = 0
    elif case == "d0":
        b.d = 0
    elif case == "d33":
        b.d = 33
    elif case == "kernel":
        b.kernel = 4
    elif case == "ard":
        b.ard = 2
    elif case == "rank_neg":
        rank = -1
    out = ctypes.c_size_t(0)
    assert lib.gp_batch_workspace_size(ctypes.byref(b), ctypes.byref(o), rank, ctypes.byref(out)) == B.GP_EINVAL
    theta = np.tile([0.5, 0.5, 0.5, 1.0, 0.1], 3)
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.gp_batch_mll_eval(ctypes.byref(b), tp, ctypes.byref(o), rank, ctypes.c_void_p(0x10000), 1 << 30, None,
                                 ctypes.c_void_p(0x3000), None) == B.GP_EINVAL


@pytest.mark.parametrize("prec,probes,rank", [("bf16x3", 8, 4), ("fp16x3", 8, 4), ("fp32", 65, 4), ("fp32", 8, 257)])
def test_batch_reports_unsupported_options(lib, prec, probes, rank):
    b, offs = _fake_batch((300, 400))
    o = B.make_options(prec, probes, 10)
    out = ctypes.c_size_t(0)
    assert lib.gp_batch_workspace_size(ctypes.byref(b), ctypes.byref(o), rank, ctypes.byref(out)) == B.GP_EUNSUPPORTED


@pytest.mark.parametrize("bad", [0.0, -1.0, float("nan")])
def test_batch_rejects_bad_theta_of_any_problem(lib, bad):
    b, offs = _fake_batch((10, 20, 5))
    o = B.make_options("fp64", 4, 10)
    theta = np.tile([0.5, 0.5, 0.5, 1.0, 0.1], 3)
    theta[2 * 5 + 4] = bad   # noise of the last problem
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.gp_batch_mll_grad(ctypes.byref(b), tp, ctypes.byref(o), 2, ctypes.c_void_p(0x10000), 1 << 30, None,
                                 ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), None) == B.GP_EINVAL
    assert lib.gp_batch_mll_grad(ctypes.byref(b), tp, ctypes.byref(o), 2, ctypes.c_void_p(0x10000), 1 << 30, None,
                                 ctypes.c_void_p(0x3000), None, None) == B.GP_EINVAL


def test_noalloc_matvec_rejects_bad_arguments_and_oversized_shapes_before_any_device_call(lib):
    theta = np.array([0.5, 0.5, 0.5, 1.0, 0.1])
    tp = theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    v, w = ctypes.c_void_p(0x5000), ctypes.c_void_p(0x6000)
    p = _fake_problem()
    f = lib.gp_khat_matvec_noalloc
    assert f(ctypes.byref(p), tp, 0, None, 4, w, None) == B.GP_EINVAL
    assert f(ctypes.byref(p), tp, 0, v, 4, None, None) == B.GP_EINVAL
    assert f(ctypes.byref(p), tp, 0, v, 0, w, None) == B.GP_EINVAL
    assert f(ctypes.byref(p), tp, 4, v, 4, w, None) == B.GP_EINVAL
    assert f(ctypes.byref(B.gp_problem(0, 0x2000, 100, 3, 0, 1)), tp, 0, v, 4, w, None) == B.GP_EINVAL
    bad = theta.copy()
    bad[4] = -1.0
    assert f(ctypes.byref(p), bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0, v, 4, w, None) == B.GP_EINVAL
    # staging arrays beyond the library's 128 MiB device array even with one column split
    big = _fake_problem(n=1_000_000)
    assert f(ctypes.byref(big), tp, 2, v, 65, w, None) == B.GP_EWORKSPACE
