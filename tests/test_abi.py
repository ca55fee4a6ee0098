"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments before touching the device (CPU-only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "entropy.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ent_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def ent():
    import paper_1801_01072_amd as ent

    return ent


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("ent_entropy_estimate", "ent_entropy_estimate_detail", "ent_power_method",
                 "ent_chebyshev_coeffs", "ent_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(ent):
    lib = ctypes.CDLL(ent.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_parameter_rules(ent):
    # Lemma 1: s = ceil(20 ln(2/delta)/eps^2)
    assert ent.probes_for(0.1, 0.05) == 7378
    # Theorem 1: m = ceil((u/l) ln(1/eps))
    assert ent.degree_taylor(1.0, 0.01, 0.1) == 231
    # Theorem 2: m = ceil(sqrt(u / (2 eps l ln(1/(1-l)))))
    import math

    want = math.ceil(math.sqrt(1.0 / (2 * 0.1 * 0.01 * math.log(1 / (1 - 0.01)))))
    assert ent.degree_chebyshev(1.0, 0.01, 0.1) == want
    # Lemma 5: q = ceil(4.82 ln(1/delta)), t = ceil(ln sqrt(4n))
    assert ent.power_trials_for(0.01) == math.ceil(4.82 * math.log(100))
    assert ent.power_iters_for(5000) == math.ceil(math.log(math.sqrt(20000)))
    assert ent.probes_for(0.0, 0.1) == -1


def test_invalid_arguments_rejected_without_device(ent):
    lib = ent._lib
    res = ent.EntResult()
    # NULL matrix
    st = lib.ent_entropy_estimate(None, 1, 10, 10, 0, None, ctypes.byref(res))
    assert st == ent.EINVAL and "NULL" in ent.last_error()
    # n < 1
    M = ent.EntMatrix(0, ent.DENSE, ent.STORE_F64, 1, 0, 1, None, None)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 10, 0, None, ctypes.byref(res)) == ent.EINVAL
    # ld < n
    M = ent.EntMatrix(10, ent.DENSE, ent.STORE_F64, 5, 0, 1, None, None)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 10, 0, None, ctypes.byref(res)) == ent.EINVAL
    # bad layout / dtype
    M = ent.EntMatrix(10, 7, ent.STORE_F64, 10, 0, 1, None, None)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 10, 0, None, ctypes.byref(res)) == ent.EINVAL
    M = ent.EntMatrix(10, ent.DENSE, 9, 10, 0, 1, None, None)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 10, 0, None, ctypes.byref(res)) == ent.EINVAL
    # CSR without index arrays
    M = ent.EntMatrix(10, ent.CSR, ent.STORE_F64, 0, 5, 1, None, None)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 10, 0, None, ctypes.byref(res)) == ent.EINVAL
    # degree, probes, method, options
    M = ent.EntMatrix(10, ent.DENSE, ent.STORE_F64, 10, 0, 1, None, None)
    for method, m, s in ((1, 0, 10), (1, 10, 0), (9, 10, 10)):
        assert lib.ent_entropy_estimate(ctypes.byref(M), method, m, s, 0, None, ctypes.byref(res)) == ent.EINVAL
    o = ent.options(precision=7)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 10, 0, ctypes.byref(o), ctypes.byref(res)) == ent.EINVAL
    o = ent.options(probe_dist=5)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 10, 0, ctypes.byref(o), ctypes.byref(res)) == ent.EINVAL
    o = ent.options(u_fixed=0.1, cutoff=0.2)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 10, 0, ctypes.byref(o), ctypes.byref(res)) == ent.EINVAL
    # output untouched on failure
    res.entropy = 123.0
    lib.ent_entropy_estimate(None, 1, 10, 10, 0, None, ctypes.byref(res))
    assert res.entropy == 123.0
    # coefficient helper argument checks
    import numpy as np

    a = np.zeros(4)
    assert lib.ent_chebyshev_coeffs(0.5, 0.4, 3, a.ctypes.data_as(ctypes.c_void_p)) == ent.EINVAL
    assert lib.ent_chebyshev_coeffs(0.0, 1.0, 0, a.ctypes.data_as(ctypes.c_void_p)) == ent.EINVAL


def test_options_defaults(ent):
    o = ent.EntOptions()
    ent._lib.ent_options_default(ctypes.byref(o))
    assert (o.power_iters, o.power_trials, o.u_factor, o.precision, o.probe_dist) == (20, 1, 6.0, ent.F64, ent.RADEMACHER)
    assert ent.version() >= 100


def test_complex_storage_rules_without_device(ent):
    lib = ent._lib
    res = ent.EntResult()
    # Hermitian storage: dense only, Taylor / Chebyshev only, estimate and power calls only
    M = ent.EntMatrix(10, ent.CSR, ent.STORE_C128, 0, 5, 1, 1, 1)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 10, 0, None, ctypes.byref(res)) == ent.EUNSUPPORTED
    M = ent.EntMatrix(10, ent.DENSE, ent.STORE_C64, 10, 0, 1, None, None)
    for method in (ent.RANDPROJ, ent.AUTO):
        assert lib.ent_entropy_estimate(ctypes.byref(M), method, 10, 10, 0, None,
                                        ctypes.byref(res)) == ent.EUNSUPPORTED
    M = ent.EntMatrix(10, ent.DENSE, ent.STORE_C128, 5, 0, 1, None, None)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 10, 0, None, ctypes.byref(res)) == ent.EINVAL
    f = (ctypes.c_float * 16)()
    M = ent.EntMatrix(10, ent.DENSE, ent.STORE_C128, 10, 0, 1, None, None)
    assert lib.ent_selector_features(ctypes.byref(M), 0, None, f, f) == ent.EUNSUPPORTED


def test_clenshaw_flag_rules_without_device(ent):
    lib = ent._lib
    res = ent.EntResult()
    M = ent.EntMatrix(10, ent.DENSE, ent.STORE_F64, 10, 0, 1, None, None)
    o = ent.options(flags=ent.FLAG_CLENSHAW)
    for method in (ent.TAYLOR, ent.AUTO):
        assert lib.ent_entropy_estimate(ctypes.byref(M), method, 10, 10, 0, ctypes.byref(o),
                                        ctypes.byref(res)) == ent.EINVAL


def test_host_array_without_device_fails_cleanly(ent):
    # a descriptor in host memory is copied to the device before anything
    # reads it; with no device here, that copy-in is a device error, the
    # result is left untouched and nothing is launched
    import numpy as np

    lib = ent._lib
    res = ent.EntResult()
    res.entropy = 123.0
    host = np.eye(8) / 8.0
    M = ent.EntMatrix(8, ent.DENSE, ent.STORE_F64, 8, 0, host.ctypes.data, None, None)
    assert lib.ent_entropy_estimate(ctypes.byref(M), 1, 10, 4, 0, None, ctypes.byref(res)) == ent.EDEVICE
    assert res.entropy == 123.0
    p1 = ctypes.c_double(7.0)
    assert lib.ent_power_method(ctypes.byref(M), 5, 1, 0, None, ctypes.byref(p1)) == ent.EDEVICE
    assert p1.value == 7.0


def test_builder_loads_without_the_package():
    """build() must work on a fresh checkout, where the library does not exist
    yet and the package's __init__ refuses to import: the builder module is
    loaded by path and never imports the package."""
    import subprocess
    import sys

    code = ("import sys, __graft_entry__ as g; b = g._load_builder(); "
            "assert callable(b.build) and b.ARCH == 'gfx950'; "
            "assert 'paper_1801_01072_amd' not in sys.modules, 'package imported'")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_flag_constants_mirror_the_header(ent):
    """The binding's ENT_FLAG_* values and the timing struct's fields are the
    header's."""
    text = open(HEADER).read()
    flags = dict((k, int(v)) for k, v in re.findall(r"\bENT_FLAG_([A-Z0-9_]+)\s*=\s*(\d+)", text))
    assert flags, "no flags parsed"
    for name, value in flags.items():
        assert getattr(ent, "FLAG_" + name) == value, name
    end = text.index("} ent_timing;")
    body = text[text.rindex("typedef struct {", 0, end):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(?:double|int32_t)\s+([a-z_]+)\s*;", body)
    assert [f for f, _ in ent.EntTiming._fields_] == fields
