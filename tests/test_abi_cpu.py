"""The C-ABI library on the host: it loads, exports every function that
include/mrtfd.h declares, its struct layouts match the Python binding, and its
parameter validation and workspace sizing work without a GPU (no compute
calls)."""
import ctypes as C
import math
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrtfd.h")


@pytest.fixture(scope="module")
def abi():
    from paper_0908_3749_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_0908_3749_amd import build_lib
        build_lib.build()
    _abi.lib()
    return _abi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mrtfd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("mrtfd_create", "mrtfd_step", "mrtfd_read_macro", "mrtfd_init_macro",
                 "mrtfd_sums", "mrtfd_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(abi):
    L = abi.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_every_declared_symbol(abi):
    assert sorted(abi.exported_names()) == declared_functions()


def test_struct_layouts_match(abi):
    ps, ss = C.c_size_t(), C.c_size_t()
    assert abi.lib().mrtfd_struct_sizes(C.byref(ps), C.byref(ss)) == 0
    assert ps.value == C.sizeof(abi.mrtfd_params)
    assert ss.value == C.sizeof(abi.mrtfd_side)


def test_status_strings(abi):
    for code in range(-6, 1):
        assert abi.lib().mrtfd_status_string(code)


def _params(prob, **kw):
    from paper_0908_3749_amd import make_params
    return make_params(prob.nx, prob.ny, prob.dx, prob.dy, prob.dt, prob.s, prob.sides, **kw)


def test_valid_params_and_workspace(abi):
    from paper_0908_3749_amd import check_params
    for prob in (synth.sod(), synth.mach_reflection(nx=256, ny=64, x0_cells=64),
                 synth.couette(nx=16, ny=64)):
        p = _params(prob)
        assert check_params(p) == (0, "")
        nbytes = abi.lib().mrtfd_workspace_bytes(C.byref(p))
        # two FP32 copies of 16 populations with ghosts, at least
        assert nbytes >= 2 * 16 * 4 * (prob.nx + 2) * (prob.ny + 2)


def test_validation_rejects_bad_params(abi):
    from paper_0908_3749_amd import check_params
    prob = synth.sod()
    p = _params(prob)
    p.dt = 1e-3  # dt * s = 50
    assert check_params(p)[0] == abi.MRTFD_ERR_UNSTABLE
    assert abi.lib().mrtfd_workspace_bytes(C.byref(p)) == 0
    p = _params(prob)
    p.dx = p.dy = 1e-4  # Courant number 6 dt / dx = 1.2
    assert check_params(p)[0] == abi.MRTFD_ERR_UNSTABLE
    p = _params(prob)
    p.nx = 2
    assert check_params(p)[0] == abi.MRTFD_ERR_ARG
    p = _params(prob)
    p.side[0].kind_lo = p.side[0].kind_hi = abi.MRTFD_BC_PERIODIC  # west periodic, east not
    assert check_params(p)[0] == abi.MRTFD_ERR_ARG
    p = _params(prob)
    p.side[0].state_lo[0] = -1.0
    assert check_params(p)[0] == abi.MRTFD_ERR_ARG
    p = _params(prob)
    p.s[6] = math.nan
    assert check_params(p)[0] == abi.MRTFD_ERR_ARG
    p = _params(prob)
    p.graph_steps = 3
    assert check_params(p)[0] == abi.MRTFD_ERR_ARG
    p = _params(prob)
    p.rows = 3
    assert check_params(p)[0] == abi.MRTFD_ERR_ARG
    p = _params(prob, collision="srt")  # the Sod rates are not all equal
    assert check_params(p)[0] == abi.MRTFD_ERR_ARG
    p = _params(prob, collision="srt")
    for k in range(4, 16):
        p.s[k] = 4e4
    assert check_params(p)[0] == abi.MRTFD_OK
    # one copy of f above 4 GiB (9000 x 8000 nodes): only the simple kernel
    # addresses it; the row kernels' 32-bit buffer offsets cannot
    p = _params(prob)
    p.nx, p.ny = 9000, 8000
    st, msg = check_params(p)
    assert st == abi.MRTFD_ERR_ARG and "4 GiB" in msg, msg
    p.kernel = abi.MRTFD_KERNEL_SIMPLE
    assert check_params(p)[0] == abi.MRTFD_OK
    p.nx, p.ny = 8192, 8063  # 64 x 8320 x 8065 B per copy: just below 2^32
    p.kernel = abi.MRTFD_KERNEL_AUTO
    assert check_params(p)[0] == abi.MRTFD_OK
    p.ny = 8064  # one more row crosses it
    st, msg = check_params(p)
    assert st == abi.MRTFD_ERR_ARG and "4 GiB" in msg, msg


def test_create_rejects_bad_workspace_without_gpu(abi):
    prob = synth.sod()
    p = _params(prob)
    ctx = C.c_void_p()
    # NULL workspace: rejected by argument checks before any HIP call
    assert abi.lib().mrtfd_create(C.byref(p), None, 0, None, C.byref(ctx)) == abi.MRTFD_ERR_ARG
    assert not ctx.value


def test_product_has_no_oracle_dependency():
    """The product package neither imports nor loads anything from oracle/."""
    pkg = os.path.join(ROOT, "paper_0908_3749_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in text.replace("the oracle", ""), fn
                assert "liboracle" not in text, fn


def test_reference_populations(abi):
    """f_ref of a reference state at rest is the equilibrium of Eq. (14)
    mapped back by M^-1 (the oracle's, independently built); no reference
    gives zeros; half a reference is rejected."""
    from oracle import core
    from paper_0908_3749_amd import check_params, ref_populations
    prob = synth.couette(nx=16, ny=64)
    p = _params(prob)
    assert list(ref_populations(p)) == [0.0] * 16
    for rho0, T0 in ((1.0, 1.0), (2.5, 0.75), (0.125, 4.0)):
        p = _params(prob, ref=(rho0, T0))
        assert check_params(p) == (0, "")
        got = ref_populations(p)
        want = core.feq_velocity(rho0, 0.0, 0.0, T0)
        assert abs(got - want).max() <= 1e-14 * abs(want).max(), (rho0, T0)
        # the conserved moments of f_ref are (rho0, 0, 0, rho0 T0)
        m = core.model()
        assert abs(m.M[:4] @ got - [rho0, 0.0, 0.0, rho0 * T0]).max() <= 1e-13
    for bad in ((1.0, 0.0), (0.0, 1.0), (-1.0, 1.0), (1.0, math.inf), (1e300, 1.0)):
        p = _params(prob, ref=bad)
        assert check_params(p)[0] == abi.MRTFD_ERR_ARG, bad


def test_screen_rejects_bad_arguments_without_gpu(abi):
    """mrtfd_screen validates its arguments before any HIP call: n < 0, a
    NULL phase array, both outputs NULL, a state with rho <= 0, T <= 0 or
    non-finite values; n = 0 does nothing."""
    p = _params(synth.sod())
    L = abi.lib()
    good = (C.c_double * 4)(1.0, 0.0, 0.0, 1.0)
    dummy = C.c_void_p(8)  # never dereferenced: every case returns before a launch
    assert L.mrtfd_screen(C.byref(p), good, dummy, 0, dummy, dummy, None) == 0
    assert L.mrtfd_screen(C.byref(p), good, dummy, -1, dummy, dummy, None) == abi.MRTFD_ERR_ARG
    assert L.mrtfd_screen(C.byref(p), good, None, 4, dummy, dummy, None) == abi.MRTFD_ERR_ARG
    assert L.mrtfd_screen(C.byref(p), good, dummy, 4, None, None, None) == abi.MRTFD_ERR_ARG
    assert L.mrtfd_screen(None, good, dummy, 4, dummy, dummy, None) == abi.MRTFD_ERR_ARG
    for bad in ((0.0, 0.0, 0.0, 1.0), (1.0, 0.0, 0.0, -1.0), (1.0, math.nan, 0.0, 1.0), (1.0, 0.0, math.inf, 1.0)):
        st = (C.c_double * 4)(*bad)
        assert L.mrtfd_screen(C.byref(p), st, dummy, 4, dummy, dummy, None) == abi.MRTFD_ERR_ARG, bad
    # dt s_k beyond 1 (refused by mrtfd_create) is what the screen is for; a bad spacing or rate is not
    from paper_0908_3749_amd import make_params
    fast = make_params(3, 3, 0.01, 0.01, 1e-5, [0.0] * 4 + [1e5] * 12, synth.sod().sides)
    fast.dt = 5e-5
    assert L.mrtfd_screen(C.byref(fast), good, dummy, 0, dummy, dummy, None) == 0
    for field, value in (("dt", 0.0), ("dx", -1.0), ("dy", math.inf)):
        q = make_params(3, 3, 0.01, 0.01, 1e-5, [0.0] * 16, synth.sod().sides)
        setattr(q, field, value)
        assert L.mrtfd_screen(C.byref(q), good, dummy, 4, dummy, dummy, None) == abi.MRTFD_ERR_ARG, field
        assert L.mrtfd_screen_sets(C.byref(q), 1, dummy, dummy, dummy, 4, dummy, dummy, None) == abi.MRTFD_ERR_ARG
    q = make_params(3, 3, 0.01, 0.01, 1e-5, [0.0] * 16, synth.sod().sides)
    q.s[7] = -1.0
    assert L.mrtfd_screen(C.byref(q), good, dummy, 4, dummy, dummy, None) == abi.MRTFD_ERR_ARG


def test_screen_sets_rejects_bad_arguments_without_gpu(abi):
    """mrtfd_screen_sets validates before any HIP call: nsets < 0, n < 0,
    nsets n of 2^31 or more, NULL inputs, both outputs NULL; nsets n = 0
    does nothing."""
    p = _params(synth.sod())
    L = abi.lib()
    d = C.c_void_p(8)  # never dereferenced: every case returns before a launch
    assert L.mrtfd_screen_sets(C.byref(p), 0, d, d, d, 5, d, d, None) == 0
    assert L.mrtfd_screen_sets(C.byref(p), 3, d, d, d, 0, d, d, None) == 0
    for args in ((-1, d, d, d, 4, d, d), (3, d, d, d, -1, d, d), (1 << 16, d, d, d, 1 << 15, d, d),
                 (3, None, d, d, 4, d, d), (3, d, None, d, 4, d, d), (3, d, d, None, 4, d, d),
                 (3, d, d, d, 4, None, None)):
        assert L.mrtfd_screen_sets(C.byref(p), *args, None) == abi.MRTFD_ERR_ARG, args
    assert L.mrtfd_screen_sets(None, 3, d, d, d, 4, d, d, None) == abi.MRTFD_ERR_ARG
