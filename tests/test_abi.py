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


def test_header_compiles_as_c_and_links(tmp_path):
    """include/dil.h is a C header (C99, pedantic, no C++ types): a C program built against it
    links to libdil.so and makes host-only calls -- the sizes, and the argument checks of the
    interactive serving calls on a NULL engine."""
    import shutil
    import subprocess
    from paper_2211_12265_amd import dilithium as dl
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    dl.load()  # the library is built
    src = tmp_path / "abi.c"
    src.write_text(r'''
#include <stdio.h>
#include "dil.h"
int main(void) {
  size_t pk = 0, sk = 0, sig = 0;
  uint64_t ticket = 0;
  int done = 0;
  if (dil_sizes(44, &pk, &sk, &sig) != DIL_OK) return 1;
  printf("%zu %zu %zu\n", pk, sk, sig);
  if (dil_server_start(NULL) != DIL_EINVAL) return 2;
  if (dil_server_submit(NULL, 0, 2, 0, NULL, 0, NULL, &ticket) != DIL_EINVAL) return 3;
  if (dil_server_poll(NULL, 1, &done, NULL, NULL) != DIL_EINVAL) return 4;
  if (dil_server_wait(NULL, 1, 0, NULL, NULL) != DIL_EINVAL) return 5;
  if (dil_server_stop(NULL) != DIL_EINVAL) return 6;
  return DIL_ETIMEDOUT == -5 ? 0 : 7;
}
''')
    exe = tmp_path / "abi"
    libdir = os.path.dirname(dl.LIB_PATH)
    res = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                          "-I", os.path.join(ROOT, "include"), str(src), dl.LIB_PATH,
                          "-Wl,-rpath," + libdir, "-o", str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.split() == ["1312", "2560", "2420"]
