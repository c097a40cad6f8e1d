"""CPU checks of the boundary: libscn.so loads and exports every entry point
include/scn.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2512_16896_amd", "libscn.so")


def declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not hdr.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", hdr)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:int\s+|const char\s*\*\s*|size_t\s+)(scn_\w+)\s*\(", src,
                            flags=re.M)
    return names


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ("scn_sample_poses", "scn_check_batch", "scn_place_step", "scn_generate_scenes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build libscn.so first (python -m paper_2512_16896_amd.build)"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2512_16896_amd import scn
    assert set(scn.EXPORTS) <= set(declared_functions())
    assert set(declared_functions()) <= set(scn.EXPORTS)


def test_status_strings_without_device():
    lib = ctypes.CDLL(LIB)
    lib.scn_status_string.restype = ctypes.c_char_p
    assert lib.scn_status_string(0) == b"ok"
    assert b"capacity" in lib.scn_status_string(-3)
    # creating a context without a device fails cleanly instead of crashing
    lib.scn_ctx_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    h = ctypes.c_void_p()
    import torch
    if not torch.cuda.is_available():
        assert lib.scn_ctx_create(ctypes.byref(h), 0) == -4
