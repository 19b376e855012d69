"""Host-side checks of the C ABI (no device needed): the library loads, it
exports every function that include/cpqr.h declares, its schedule engine
agrees with the oracle's independent schedule, and its argument checks
return the documented status codes."""
import os
import re
import ctypes

import numpy as np
import pytest

import oracle as O
import paper_2503_18759_amd as P
from paper_2503_18759_amd import cpqr as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "cpqr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cpqr_[a-z_0-9]+)\s*\(", src)))


def test_library_loads_and_exports_header_symbols():
    lib = ctypes.CDLL(C.LIB_PATH)
    names = _header_functions()
    assert "cpqr_als_qr" in names and "cpqr_schedule" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in cpqr.h but not exported"
    assert sorted(C.EXPORTS) == names


def test_status_strings():
    L = C.load_library()
    for code, name in [(0, "CPQR_OK"), (-1, "CPQR_EINVAL"), (-2, "CPQR_EUNSUPPORTED"),
                       (-5, "CPQR_ERANKDEF"), (-6, "CPQR_ENONFINITE")]:
        assert L.cpqr_status_string(code).decode() == name


def _oracle_steps(N, tree, sweeps):
    out = []
    for steps in O.tree_schedule(N, tree, sweeps):
        for s in steps:
            if s[0] == "ttm":
                out.append((0, sum(1 << m for m in s[1]), s[2]))
            else:
                out.append((1, 0, s[1]))
    return out


@pytest.mark.parametrize("N", [3, 4, 5, 6, 7])
@pytest.mark.parametrize("tree", ["none", "standard", "restructured"])
def test_engine_schedule_equals_oracle_schedule(N, tree):
    orders, steps, poly = P.schedule(N, tree, 8)
    assert steps == _oracle_steps(N, tree, 8)
    for k in range(8):
        assert orders[k] == O.sweep_order(N, tree, k + 1)
    assert poly == O.schedule_flops(O.tree_schedule(N, tree, 8), N)


def test_engine_three_sweep_cost_matches_table3():
    # Table 3, restructured: 8 I1I2I3 R + 4 I1I2 R^2 + 8 I1I3 R^2 + 6 I2I3 R^2
    _, _, poly = P.schedule(3, "restructured", 3)
    assert poly == {((0, 1, 2), 1): 8, ((0, 1), 2): 4, ((0, 2), 2): 8, ((1, 2), 2): 6}


def test_schedule_rejects_bad_arguments():
    L = C.load_library()
    n = ctypes.c_int(0)
    assert L.cpqr_schedule(1, 2, 3, None, None, 0, ctypes.byref(n), None) == C.EINVAL
    assert L.cpqr_schedule(3, 7, 3, None, None, 0, ctypes.byref(n), None) == C.EINVAL
    assert L.cpqr_schedule(3, 2, 0, None, None, 0, ctypes.byref(n), None) == C.EINVAL
    assert L.cpqr_schedule(3, 2, 3, None, None, 0, ctypes.byref(n), None) == C.OK
    steps = (ctypes.c_int * 3)()
    assert L.cpqr_schedule(3, 2, 3, None, steps, 1, ctypes.byref(n), None) == C.EINVAL


@pytest.mark.parametrize("kwargs,expect", [
    (dict(dims=[40, 40, 40], rank=5, dtype="f64", prec="fp64"), C.OK),
    (dict(dims=[256, 256, 256], rank=32), C.OK),
    (dict(dims=[40] * 5, rank=16), C.OK),
    (dict(dims=[40, 40, 4], rank=5), C.OK),                    # I_n < R: compact factor QR
    (dict(dims=[3, 40, 2, 30], rank=8), C.OK),                 # two modes below the rank
    (dict(dims=[2, 2, 40], rank=5), C.EUNSUPPORTED),           # Z_3 has 2*2 < 5 nonzero rows
    (dict(dims=[1, 40], rank=2, tree="none"), C.EUNSUPPORTED),  # order 2: Z_2 = R_1 has 1 row
    (dict(dims=[40, 40, 40], rank=33), C.EUNSUPPORTED),        # rank above this build's limit
    (dict(dims=[600, 40, 40], rank=5), C.OK),                  # mode above 512: factor TSQR
    (dict(dims=[2048, 256, 256], rank=32), C.OK),              # Density-sized
    (dict(dims=[8192, 40, 40], rank=32), C.OK),                # largest two-level factor TSQR at R 32
    (dict(dims=[8193, 40, 40], rank=32), C.EUNSUPPORTED),
    (dict(dims=[40] * 5, rank=32), C.EUNSUPPORTED),            # order 5 beyond the Z QR at rank 32
    (dict(dims=[100] * 4, rank=30), C.OK),                     # Z_n 27,000 x 30: nested QR only
    (dict(dims=[100] * 4, rank=30, flags=0x8), C.EUNSUPPORTED),  # ... beyond the dense TSQR
    (dict(dims=[6] * 6, rank=16), C.OK),                       # order 6, Z_n of 16^5 rows
    (dict(dims=[6] * 7, rank=16), C.EUNSUPPORTED),             # order 7 beyond the Z QR at rank 16
    (dict(dims=[40, 40, 40], rank=0), C.EINVAL),
    (dict(dims=[40, 40, 40], rank=5, prec="fp64"), C.EINVAL),  # f32 data with fp64 precision
    (dict(dims=[40, 40, 40], rank=5, dtype="f64"), C.EINVAL),  # f64 data with fp32 precision
    (dict(dims=[40, 40, 40], rank=5, iters=0), C.EINVAL),
    (dict(dims=[40, 40, 40], rank=5, tol=-1.0), C.EINVAL),
    (dict(dims=[40, 40], rank=5, tree="restructured"), C.EINVAL),
    (dict(dims=[40, 40], rank=5, tree="none"), C.OK),
    (dict(dims=[40, 40, 40], rank=5, data_ptr=0), C.EINVAL),
    (dict(dims=[40, 40, 40], rank=5, raw={"tree": 5}), C.EINVAL),
    (dict(dims=[40, 40, 40], rank=5, raw={"prec": 3}), C.EINVAL),
    (dict(dims=[40, 40, 40], rank=5, raw={"extrapolate": 4}), C.EINVAL),
    (dict(dims=[40, 40, 40], rank=5, extrapolate="learned"), C.EINVAL),   # learned needs mlp_weights
    (dict(dims=[40, 40, 40], rank=5, extrapolate="learned", mlp_weights=True), C.OK),
    (dict(dims=[40, 40, 40], rank=5, raw={"null_init": True}), C.OK),      # seeded N(0,1) factors
    (dict(dims=[40, 40, 40], rank=5, flags=0x10 | 0x2), C.EINVAL),        # phase and kernel timing
    (dict(dims=[40, 40, 40], rank=5, flags=0x10), C.OK),
    (dict(dims=[40, 40, 40], rank=5, raw={"null_init_k": 1}), C.EINVAL),
    (dict(dims=[40, 40, 40], rank=5, raw={"null_dims": True}), C.EINVAL),
    (dict(dims=[40, 0, 40], rank=5), C.EINVAL),
    (dict(dims=[40] * 8, rank=2), C.EINVAL),                  # order above the limit
])
def test_argument_checks(kwargs, expect):
    kw = dict(kwargs)
    dims, rank = kw.pop("dims"), kw.pop("rank")
    assert P.check_args(dims, rank, **kw) == expect


def test_python_layer_fails_loudly_without_library(tmp_path):
    with pytest.raises(RuntimeError, match="not found"):
        C._lib_saved = C._lib
        try:
            C._lib = None
            C.load_library(str(tmp_path / "missing.so"))
        finally:
            C._lib = C._lib_saved


def test_tune_cache_file_format():
    """The TTM tuning file (include/cpqr.h): entries for the matching device,
    none for another, and malformed files rejected."""
    import paper_2503_18759_amd as P
    P.load_library()
    good = ('{"format": 1, "device": "gfx950:256",\n "entries": {\n'
            '  "ttm/p1/L1/I256/S65536/R32": [1, 2],\n  "ttmb/p1/nb1/kc/5/0123456789abcdef": [4, 1]\n }\n}\n')
    assert P.tune_cache_check(good, "gfx950:256") == 2
    assert P.tune_cache_check(good, "gfx942:304") == 0
    assert P.tune_cache_check('{"format": 1, "device": "x", "entries": {}}', "x") == 0
    bad = [good.replace("[1, 2]", "[3, 2]"),          # K split outside 1/2/4
           good.replace("[1, 2]", "[1, 5]"),          # workgroups per CU outside 0..2
           good.replace('"format": 1', '"format": 2'),
           good.replace('"device": "gfx950:256",', ""),
           good.replace("[4, 1]", "[4 1]"),
           good[:-3], "", "[]", '{"format": 1, "device": "x", "other": 1}']
    for b in bad:
        with pytest.raises(P.CpqrError):
            P.tune_cache_check(b, "gfx950:256")
