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


def test_nonfinite_status_string():
    lib = ctypes.CDLL(LIB)
    lib.scn_status_string.restype = ctypes.c_char_p
    assert b"non-finite" in lib.scn_status_string(-6)


def test_workspace_bytes_on_the_host():
    """scn_workspace_bytes is host arithmetic on the sizes (no device): the
    longest-first order of n scenes, the network's hidden activations, and
    the learned generation's buffers (at least its logits and features)."""
    from paper_2512_16896_amd import scn
    al = lambda v: (v + 255) // 256 * 256
    b = scn._Batch()
    b.n_scenes, b.n_objects = 1000, 20000
    n = ctypes.c_size_t()
    assert scn.lib().scn_workspace_bytes(scn.WS_GENERATE, ctypes.byref(b), None, 0, 0,
                                         ctypes.byref(n)) == 0
    assert n.value == al(4 * 1000) + al(4 * 257)
    net = scn.Mlp()
    for l, d in enumerate((4128, 512, 512, 512, 4096)):
        net.dims[l] = d
    assert scn.lib().scn_workspace_bytes(scn.WS_MLP_FORWARD, None, ctypes.byref(net), 96, 0,
                                         ctypes.byref(n)) == 0
    assert n.value == 3 * al(96 * 512 * 2)
    assert scn.lib().scn_workspace_bytes(scn.WS_MLP_TRAIN, None, ctypes.byref(net), 256, 0,
                                         ctypes.byref(n)) == 0
    grads = sum(al(4 * o * i) + al(4 * o) for i, o in ((4128, 512), (512, 512), (512, 512),
                                                        (512, 4096)))
    assert n.value > grads
    assert scn.lib().scn_workspace_bytes(scn.WS_GENERATE_LEARNED, ctypes.byref(b),
                                         ctypes.byref(net), 0, 64, ctypes.byref(n)) == 0
    assert n.value >= 1000 * (4096 * 4 + 4128 * 2 + 4096 * 4 + 64 * 4) + 20000 * 32 * 4
    # bad arguments are refused without a device
    assert scn.lib().scn_workspace_bytes(99, ctypes.byref(b), None, 0, 0, ctypes.byref(n)) == -1
    assert scn.lib().scn_workspace_bytes(scn.WS_GENERATE_LEARNED, ctypes.byref(b),
                                         ctypes.byref(net), 0, 0, ctypes.byref(n)) == -1
    assert scn.lib().scn_set_workspace(None, None, 0) == -1
