"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function that include/dil.h declares, and answers the pure host calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(dil_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_2211_12265_amd import dilithium as dl
    lib = dl.load()
    decl = _declared()
    assert len(decl) >= 12
    missing = [n for n in decl if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(dl.EXPORTS) == decl


def test_sizes_and_invalid_level():
    from paper_2211_12265_amd import dilithium as dl
    assert dl.sizes(2) == (1312, 2528, 2420)
    assert dl.sizes(3) == (1952, 4000, 3293)
    assert dl.sizes(5) == (2592, 4864, 4595)
    with pytest.raises(dl.DilError):
        dl.sizes(4)


def test_null_context_rejected():
    from paper_2211_12265_amd import dilithium as dl
    lib = dl.load()
    assert lib.dil_sign_batch(None, 2, None, None, None, None, None, 0, None) == dl.DIL_EINVAL
    assert lib.dil_ctx_destroy(None) == dl.DIL_EINVAL
