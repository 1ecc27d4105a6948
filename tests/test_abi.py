"""The C-ABI library loads and exports every entry point include/pmf.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmf.h")
LIB = os.path.join(ROOT, "paper_2412_07240_amd", "libpmf.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pmf_[a-z_]+)\s*\(", text)))


def test_header_declares_the_core_calls():
    names = declared()
    for core in ("pmf_create", "pmf_predict", "pmf_update", "pmf_moments", "pmf_batch_step"):
        assert core in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libpmf.so not built (run __graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    from paper_2412_07240_amd import binding
    assert set(declared()) <= set(binding.EXPORTED)
    binding.lib()


def test_struct_layouts_match_header_sizes():
    """ctypes mirrors of the public structs have the C layout (sizes from a
    host compile of the header)."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    from paper_2412_07240_amd import binding
    src = ('#include "pmf.h"\n#include <stdio.h>\nint main(){printf("%zu %zu %zu %zu %zu %zu\\n",'
           'sizeof(pmf_model),sizeof(pmf_prior),sizeof(pmf_state_header),sizeof(pmf_completion),'
           'sizeof(pmf_server_stats),sizeof(pmf_allocator));return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    assert [int(x) for x in out] == [ctypes.sizeof(binding.pmf_model), ctypes.sizeof(binding.pmf_prior),
                                     ctypes.sizeof(binding.pmf_state_header),
                                     ctypes.sizeof(binding.pmf_completion),
                                     ctypes.sizeof(binding.pmf_server_stats),
                                     ctypes.sizeof(binding.pmf_allocator)]
