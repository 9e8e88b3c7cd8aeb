"""The C interface without a GPU: the library loads and exports every
function that include/*.h declares; the binding declares the same set."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2509_05090_amd", "libctm.so")


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(ctm_[a-z_0-9]+)\s*\(", text))
    return names


def test_headers_declare_the_boundary():
    names = declared_functions()
    for required in ("ctm_init", "ctm_step", "ctm_converge", "ctm_energy", "ctm_grad",
                     "ctm_free", "ctm_last_error", "ctm_symmetrize", "ctm_spectrum"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libctm.so not built"
    lib = ctypes.CDLL(LIB)
    for name in sorted(declared_functions()):
        assert hasattr(lib, name), name


def test_binding_covers_the_exports():
    from paper_2509_05090_amd import ctm
    assert set(ctm.EXPORTS) == declared_functions()


def test_argument_errors_without_device_work():
    """Calls rejected before any device work: null context / bad config."""
    from paper_2509_05090_amd import ctm
    lib = ctm._lib
    assert lib.ctm_step(None, 1, None) == ctm.CTM_EINVAL
    assert lib.ctm_query(None, None, None, None) == ctm.CTM_EINVAL
    assert "null" in ctm.last_error()
    h = ctypes.c_void_p()
    bad = ctm._Config(2, 0, 8, 0, 0)
    assert lib.ctm_init(ctypes.byref(h), ctypes.byref(bad), ctypes.c_void_p(8),
                        ctypes.c_void_p(8), None) == ctm.CTM_EINVAL
    evd = ctm._Config(2, 10, 100, 1, 0)  # eigendecomposition projector needs chi D^2 <= 8192
    assert lib.ctm_init(ctypes.byref(h), ctypes.byref(evd), ctypes.c_void_p(8),
                        ctypes.c_void_p(8), None) == ctm.CTM_EINVAL
    assert lib.ctm_symmetrize(None, None, 2, 2, None) == ctm.CTM_EINVAL
    assert lib.ctm_grad(None, None, 0, 1e-12, 10, None, None, None) == ctm.CTM_EINVAL
    lib.ctm_free(None)
