"""The C-ABI library loads on the CPU and exports every declared entry point.

No compute call is made here (no GPU in this environment)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2010_00881_amd", "libfcm.so")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fcm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fcm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ["fcm_setup", "fcm_vcycle", "fcm_pcg_solve", "fcm_serve_submit"]:
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfcm.so not built")
def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    from paper_2010_00881_amd import fcm
    assert set(fcm.SIGNATURES) == set(declared_symbols())
    lib.fcm_status_string.restype = ctypes.c_char_p
    assert lib.fcm_status_string(0) == b"ok"
    assert lib.fcm_status_string(-4) == b"matrix not positive definite"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfcm.so not built")
def test_struct_layouts_match_header():
    import ctypes
    from paper_2010_00881_amd import fcm
    # the C structs are plain; sizes follow the C alignment rules for x86-64
    # 7 fields, then use_graphs, autotune, coarse and coarse_dense_max
    assert ctypes.sizeof(fcm.Options) == 64
    assert ctypes.sizeof(fcm.SolveInfo) == 56
    assert ctypes.sizeof(fcm.Problem) == 280     # ..., surf_n[2], space, psi, trig_src, trig_dir
    assert ctypes.sizeof(fcm.Stats) == 64
    assert ctypes.sizeof(fcm.ServerOpts) == 16


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfcm.so not built")
@pytest.mark.parametrize("change, opt, msg", [
    ({"dim": 4}, {}, "dim must be 2 or 3"),
    ({"refine_levels": 5}, {}, "refine_levels must be in 0..4"),
    ({"refine_levels": 1}, {"smoother": "elementwise", "omega": 2.0 / 15.0}, "patchwise"),
    ({"refine_levels": 1, "quad_depth": 4}, {}, "quad_depth must be <= 3"),
    ({"refine_levels": 0}, {}, "needs refine_levels > 0"),
    ({"geom": 0}, {}, "ball-interior geometry"),
    ({"alpha": 0.0}, {}, "alpha must be in (0,1]"),
    ({"p": 9}, {}, "p must be in 1.."),
    ({"refine_levels": 1}, {"coarse": "hmg"}, "coarse level is solved exactly"),
    ({"refine_levels": 1, "space": "trunk"}, {}, "tensor-product space only"),
    ({"refine_levels": 0, "beta": 0.0}, {"coarse": "hmg", "coarse_dense_max": 9000},
     "coarse_dense_max must be in 0..8192"),
])
def test_setup_rejects_invalid_problems_before_any_device_call(change, opt, msg):
    """fcm_setup validates the problem on the host and returns FCM_ERR_ARG with
    a description before it touches the device (so this runs without a GPU)."""
    import ctypes
    import fcm_inputs as fi
    from paper_2010_00881_amd import fcm
    d, o = fi.sphere_multilevel(0, n=4, k=1, p=2)
    d.update(change)
    pd = fcm._ProblemData(d)
    opts = fcm.make_options({**o, "precision": "fp64", **opt})
    h = ctypes.c_void_p()
    st = fcm.lib().fcm_setup(ctypes.byref(pd.struct), ctypes.byref(opts), None, ctypes.byref(h))
    assert st == -1 and not h.value
    assert msg in fcm.lib().fcm_last_error().decode()
