"""The C-ABI library loads and exports every entry point include/spd.h declares;
argument validation happens on the host before any device work (so these
calls are safe without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spd.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(spd_[a-z_]+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1405_4644_amd as spd
    if not os.path.exists(spd.LIB_PATH):
        pytest.fail("libspd.so is not built (python -m paper_1405_4644_amd.build)")
    return spd.load()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("spd_factor", "spd_factor_import", "spd_solve", "spd_refine", "spd_solve_batched", "spd_factor_destroy",
                     "spd_status_str", "spd_cg_prepare", "spd_cg_refine", "spd_cg_destroy", "spd_cg_opts_default"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    import paper_1405_4644_amd as spd
    bound = {name for name, _, _ in spd._SIGS}
    assert set(_declared()) == bound


def test_status_strings(lib):
    import paper_1405_4644_amd as spd
    assert spd.status_str(0) == "SPD_OK"
    assert spd.status_str(2) == "SPD_ERR_NOT_SPD"
    assert spd.status_str(3) == "SPD_ERR_NO_CONVERGENCE"
    assert spd.status_str(99) == "SPD_ERR_UNKNOWN"


def test_defaults(lib):
    import paper_1405_4644_amd as spd
    o = spd.default_opts()
    assert (o.tol, o.max_iter, o.fallback, o.equilibrate, o.theta) == (1e-14, 10, 1, 1, 0.1)


def test_invalid_arguments_rejected_on_host(lib):
    import paper_1405_4644_amd as spd
    info = C.c_int64()
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.spd_factor(None, -1, 1, 2, None, None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG
    assert lib.spd_factor(fake, 10, 5, 2, None, None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG  # lda < n
    assert lib.spd_factor(None, 10, 10, 2, None, None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG  # A NULL
    assert lib.spd_factor(fake, 10, 10, 7, None, None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG  # prec
    assert lib.spd_factor(fake, 10, 10, 2, None, None, None, C.byref(info)) == spd.ERR_INVALID_ARG  # F NULL
    bad = spd.default_opts(theta=0.0)
    assert lib.spd_factor(fake, 10, 10, 2, C.byref(bad), None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG
    bad = spd.default_opts(max_iter=-1)
    assert lib.spd_factor(fake, 10, 10, 2, C.byref(bad), None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG
    assert lib.spd_solve(None, fake, 10, 1, fake, 10, None) == spd.ERR_INVALID_ARG
    rep = spd.Report()
    assert lib.spd_refine(None, fake, 10, fake, 10, 1, fake, 10, None, C.byref(rep), None) == spd.ERR_INVALID_ARG
    assert lib.spd_residual(fake, 10, 9, fake, 10, fake, 10, 1, None, 10, None, None) == spd.ERR_INVALID_ARG
    assert lib.spd_residual(None, 10, 10, fake, 10, fake, 10, 1, None, 10, None, None) == spd.ERR_INVALID_ARG
    assert lib.spd_solve_batched(-1, None, None, None, None, None, None, None, None, None, None,
                                 None) == spd.ERR_INVALID_ARG
    assert lib.spd_solve_batched(0, None, None, None, None, None, None, None, None, None, None, None) == spd.OK
    # non-empty batch with a missing array: rejected before any device work
    assert lib.spd_solve_batched(3, fake, fake, fake, fake, None, fake, fake, fake, None, fake,
                                 None) == spd.ERR_INVALID_ARG
    # factor import: binary32 / binary64 only, ldl >= n, L and F present
    assert lib.spd_factor_import(fake, 10, 5, 3, None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG
    assert lib.spd_factor_import(None, 10, 10, 3, None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG
    assert lib.spd_factor_import(fake, 10, 10, 1, None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG
    assert lib.spd_factor_import(fake, 10, 10, 0, None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG
    assert lib.spd_factor_import(fake, -1, 10, 3, None, C.byref(h), C.byref(info)) == spd.ERR_INVALID_ARG
    assert lib.spd_factor_import(fake, 10, 10, 3, None, None, C.byref(info)) == spd.ERR_INVALID_ARG
    assert lib.spd_factor_query(None, None, None, None) == spd.ERR_INVALID_ARG
    assert lib.spd_factor_export(None, None, 1, None, None, None) == spd.ERR_INVALID_ARG
    lib.spd_factor_destroy(None)  # no-op
    # CG (Algorithm 2): handle, sizes, pointers; band limit; defaults
    hc = C.c_void_p()
    assert lib.spd_cg_prepare(fake, 10, 10, -1, None, None) == spd.ERR_INVALID_ARG
    assert lib.spd_cg_prepare(fake, -1, 10, -1, None, C.byref(hc)) == spd.ERR_INVALID_ARG
    assert lib.spd_cg_prepare(fake, 10, 5, -1, None, C.byref(hc)) == spd.ERR_INVALID_ARG
    assert lib.spd_cg_prepare(None, 10, 10, -1, None, C.byref(hc)) == spd.ERR_INVALID_ARG
    assert lib.spd_cg_prepare(fake, 10000, 10000, 5000, None, C.byref(hc)) == spd.ERR_UNSUPPORTED
    assert not hc
    rep = spd.Report()
    assert lib.spd_cg_refine(None, fake, 10, fake, 10, 1, fake, 10, None, C.byref(rep), None) == spd.ERR_INVALID_ARG
    lib.spd_cg_destroy(None)  # no-op
    o = spd.cg_default_opts()
    assert (o.tol, o.inner_tol, o.max_outer, o.max_inner) == (1e-14, 1e-6, 30, 2000)


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_1405_4644_amd as spd
    saved = spd._lib
    try:
        spd._lib = None
        with pytest.raises(RuntimeError):
            spd.load(str(tmp_path / "missing.so"))
    finally:
        spd._lib = saved


def test_wait_limit_argument_checks(lib):
    import paper_1405_4644_amd as spd
    assert lib.spd_factor_set_wait_limit(None, 1.0) == spd.ERR_INVALID_ARG


def test_noalloc_residual_rejects_sizes_beyond_its_array(lib):
    # checked before any device work: n = 20000 with 2 right-hand sides needs
    # more partial sums than the static array holds
    import paper_1405_4644_amd as spd
    fake = C.c_void_p(0x1000)
    assert lib.spd_residual_noalloc(fake, 20000, 20000, fake, 20000, fake, 20000, 2, fake, 20000, None,
                                    None) == spd.ERR_INVALID_ARG
    assert lib.spd_residual_noalloc(fake, 10, 5, fake, 10, fake, 10, 1, fake, 10, None, None) == spd.ERR_INVALID_ARG


def test_autotune_argument_checks(lib):
    import paper_1405_4644_amd as spd
    r = spd.TuneResult()
    assert lib.spd_autotune(0, 2, None, C.byref(r)) == spd.ERR_INVALID_ARG
    assert lib.spd_autotune(1024, 7, None, C.byref(r)) == spd.ERR_INVALID_ARG
    assert lib.spd_autotune(1024, 2, None, None) == spd.ERR_INVALID_ARG


def test_one_hip_runtime_per_process():
    # torch carries its own HIP runtime under the same soname; loading the
    # library first must not map a second one next to it (torch's streams and
    # allocations would then be foreign to the library).  A fresh interpreter,
    # the library loaded before anything imports torch; no device call.
    import subprocess
    import sys
    code = ("import paper_1405_4644_amd as spd; spd.load(); import torch; "
            "m = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1", out.stdout
