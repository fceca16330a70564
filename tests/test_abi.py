"""The C-ABI library loads and exports every symbol declared in include/ifeti.h (CPU only)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ifeti.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(ifeti_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2308_11371_amd import ifeti
    if not os.path.exists(ifeti.LIB_PATH):
        from paper_2308_11371_amd import build
        build.build(verbose=False)
    return ifeti.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_2308_11371_amd import ifeti
    assert sorted(ifeti.EXPORTED) == _declared()


@pytest.mark.parametrize("field,value", [("dim", 4), ("n_el", 0), ("degree", 3), ("nu", 0.5),
                                         ("dirichlet_mask", 0), ("load_face", 9)])
def test_invalid_descriptions_rejected_without_gpu(lib, field, value):
    """ifeti_create validates its description before any device call."""
    import ctypes
    from paper_2308_11371_amd import ifeti
    d = ifeti.LatticeDesc(2, 2, 2, 1, 3, 2, 1.0, 1.0, 1e-3, 0.3, 0.0, 1, 1)
    setattr(d, field, value)
    h = ctypes.c_void_p()
    st = lib.ifeti_create(ctypes.byref(h), ctypes.byref(d), None)
    assert st == ifeti.IFETI_EINVAL
    assert lib.ifeti_last_error().decode()
    assert not h.value


def test_null_arguments_rejected(lib):
    from paper_2308_11371_amd import ifeti
    assert lib.ifeti_create(None, None, None) == ifeti.IFETI_EINVAL
    assert lib.ifeti_get_sizes(None, None) == ifeti.IFETI_EINVAL
    assert lib.ifeti_apply_F(None, None, None, 1) == ifeti.IFETI_EINVAL
