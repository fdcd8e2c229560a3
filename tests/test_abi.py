"""The C ABI library loads, exports every symbol include/rt3d.h declares, and
rejects bad arguments on the host before touching a GPU (no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rt3d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rt3d_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1905_06700_amd import rt3d
    return rt3d.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    from paper_1905_06700_amd import rt3d
    assert sorted(rt3d.EXPORTS) == sorted(names)


def test_struct_sizes_match_header(L):
    from paper_1905_06700_amd import rt3d
    p = rt3d.default_params()
    assert p.struct_size == C.sizeof(rt3d.Params)
    assert p.n_iter == 20 and p.k_max == 4 and p.beta_t == 0.5 and p.denoiser == rt3d.DENOISE_APSS


def test_create_rejects_bad_arguments_on_host(L):
    from paper_1905_06700_amd import rt3d
    p = rt3d.default_params()
    h = C.c_void_p()

    def create(irf, bins, origin=-1, params=p):
        arr = (C.c_double * max(1, len(irf)))(*irf)
        return L.rt3d_create(arr, len(irf), origin, bins, C.byref(params), C.byref(h))

    assert create([0.0, 0.0], 100) == rt3d.E_INVALID            # zero sum
    assert create([1.0, -1.0], 100) == rt3d.E_INVALID           # negative sample
    assert create([1.0, float("nan")], 100) == rt3d.E_INVALID
    assert create([1.0] * 11, 10) == rt3d.E_INVALID             # longer than the histogram
    assert create([1.0], 70000) == rt3d.E_INVALID               # bins above 65535
    assert create([1.0, 2.0], 100, origin=2) == rt3d.E_INVALID  # origin outside the IRF
    bad = rt3d.default_params(k_max=5)
    assert create([1.0], 100, params=bad) == rt3d.E_INVALID
    bad = rt3d.default_params(h_apss=0.0)
    assert create([1.0], 100, params=bad) == rt3d.E_INVALID
    bad = rt3d.default_params(denoiser=7)
    assert create([1.0], 100, params=bad) == rt3d.E_UNSUPPORTED
    bad = rt3d.default_params()
    bad.struct_size = 8
    assert create([1.0], 100, params=bad) == rt3d.E_INVALID
    assert h.value is None


def test_null_context_calls_are_safe(L):
    from paper_1905_06700_amd import rt3d
    L.rt3d_destroy(None)
    assert L.rt3d_last_error(None) == b"null context"
    assert L.rt3d_query(None, None, None) == rt3d.E_INVALID
    assert L.rt3d_workspace_bytes(None, 1, 1, 1, 1) == 0
