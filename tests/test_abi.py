"""The C interface: the library loads without a GPU, exports every entry point that
include/*.h declares, and its host-side checks behave as documented."""
import glob
import os
import re

import numpy as np
import pytest

from paper_2603_19439_amd import grest as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grest.h")
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions(headers=HEADERS):
    names = set()
    for h in headers:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(grest_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions([HEADER])
    for required in ["grest_create", "grest_set_pairs", "grest_init_pairs", "grest_update", "grest_sync",
                     "grest_get", "grest_destroy", "grest_validate_changes", "grest_strerror"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = G.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    bound = {name for name, _, _ in G._SIGS}
    assert set(declared_functions()) <= bound


def test_abi_version_and_strerror():
    lib = G.lib()
    assert lib.grest_abi_version() == 1
    assert lib.grest_strerror(0) == b"ok"
    assert lib.grest_strerror(1).startswith(b"invalid")


@pytest.mark.parametrize("case,ok", [
    (dict(n=5, s=0, i=[0, 1], j=[1, 2], g=[1, -1]), True),
    (dict(n=5, s=2, i=[0, 4], j=[5, 6], g=[1, 1]), True),
    (dict(n=5, s=0, i=[1], j=[1], g=[1]), False),        # self-loop
    (dict(n=5, s=0, i=[2], j=[1], g=[1]), False),        # i > j
    (dict(n=5, s=0, i=[0], j=[5], g=[1]), False),        # out of range
    (dict(n=5, s=1, i=[0], j=[5], g=[-1]), False),       # delete on an appended node
    (dict(n=5, s=0, i=[0, 0], j=[3, 3], g=[1, 1]), False),  # duplicate
    (dict(n=5, s=0, i=[0], j=[3], g=[2]), False),        # bad sign
    (dict(n=5, s=0, i=[], j=[], g=[]), True),            # empty update
])
def test_host_validation(case, ok):
    assert G.validate_changes(case["n"], case["s"], case["i"], case["j"], case["g"]) == ok


def test_create_without_device_or_with_bad_args_fails_cleanly():
    rp = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    with pytest.raises(G.GrestError) as e:
        G.State(rp, col, k=5)  # k >= n
    assert e.value.status in (G.EINVAL, G.ENODEV)
    bad = np.array([1, 1], dtype=np.int32)  # self-loop in row 1
    with pytest.raises(G.GrestError):
        G.State(rp, bad, k=1)


def _checkpoint(es=8, prec=0, proj=0, has_pairs=0, graph_free=0, ax_valid=0, magic=b"GRESTCK1", n=3, m=2,
                truncate=0):
    """A checkpoint buffer of the layout grest_save writes (header, then the CSR), for a
    3-node graph with one edge and no pairs."""
    import struct
    cfg = struct.pack("<8id", 1, 2, 0, 0, 0, prec, 0, proj, 0.0)  # k=1, G-REST2, adjacency
    head = struct.pack("<8sii", magic, 1, es) + cfg + struct.pack("<qqqq", n, m, n + 1, m + 1024) + \
        struct.pack("<iiii", has_pairs, graph_free, ax_valid, 0)
    body = b""
    if not graph_free:
        body = np.array([0, 1, 2, 2], dtype=np.int64).tobytes() + np.array([1, 0], dtype=np.int32).tobytes()
    buf = head + body
    return buf[:len(buf) - truncate] if truncate else buf


@pytest.mark.parametrize("kw,valid", [
    (dict(), True),
    (dict(es=4), False),                      # FP32 elements for an FP64 configuration
    (dict(magic=b"GRESTCKX"), False),         # not a checkpoint
    (dict(truncate=4), False),                # truncated
    (dict(graph_free=1), False),              # a released graph for the exact form
    (dict(ax_valid=1), False),                # a kept product without pairs
    (dict(proj=1, ax_valid=0, graph_free=0), True),
])
def test_checkpoint_header_checks_on_the_host(kw, valid):
    """grest_load checks a checkpoint on the host before any device call: malformed buffers
    are EINVAL; a well-formed one reaches the device (ENODEV without a GPU)."""
    import ctypes as C
    lib = G.lib()
    buf = _checkpoint(**kw)
    cbuf = C.create_string_buffer(buf, len(buf))
    out = C.c_void_p()
    rc = lib.grest_load(cbuf, len(buf), None, C.byref(out))
    if valid:
        assert rc in (G.OK, G.ENODEV), rc
        if rc == G.OK:
            lib.grest_destroy(out)
    else:
        assert rc == G.EINVAL, rc


@pytest.mark.parametrize("n,w,ldz,ldy", [(0, 8, 8, 8), (2**31, 8, 8, 8), (10, 6, 8, 8), (10, 8, 6, 8),
                                         (10, 8, 8, 10), (10, 8, 8, 8)])
def test_calib_gather_rejects_bad_arguments_on_the_host(n, w, ldz, ldy):
    # every case is refused before a launch (the last for its null buffers)
    rc = G.lib().grest_calib_gather(n, None, None, ldz, w, None, ldy, 1, None)
    assert rc == 1
