"""CPU-side checks of the C ABI: the library loads, exports every entry point
include/lt.h declares, and sizes its side state as the method prescribes
(no compute call; these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2609_32920_amd import lt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lt.LIB_PATH):
        pytest.fail("liblt.so is not built; run __graft_entry__.build()")
    return lt.library()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lt_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_paper_entry_points():
    names = declared_functions()
    for n in ("lt_scene_upload", "lt_trace", "lt_backward_naive", "lt_backward_reslrb", "lt_backward_lrb3",
              "lt_backward_lrb2"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert names
    for n in names:
        assert hasattr(lib, n), n
    assert set(lt.exported_symbols()) == set(names)


def _args(n, d, flags):
    a = lt.TraceArgs()
    a.seed, a.n_paths, a.max_depth, a.flags = 1, n, d, flags
    return a


def test_side_state_linear_for_tape_flat_for_replay(lib):
    n = 1 << 22
    tape = [lib.lt_side_state_bytes(None, C.byref(_args(n, d, lt.RECORD_TAPE))) for d in (8, 16, 32)]
    res = [lib.lt_side_state_bytes(None, C.byref(_args(n, d, lt.RECORD_RESERVOIR))) for d in (8, 16, 32)]
    none = [lib.lt_side_state_bytes(None, C.byref(_args(n, d, 0))) for d in (8, 16, 32)]
    # naive tape: one 32-byte record per (vertex, path) plus one length per path
    base = [t - 32 * n * d for t, d in zip(tape, (8, 16, 32))]
    assert base[0] == base[1] == base[2] and base[0] >= 4 * n
    # ResLRB: one 32-byte record per path, independent of depth
    assert res[0] == res[1] == res[2] == 32 * n
    # LRB-3: nothing
    assert none == [0, 0, 0]
    # buffered two-pass: a 16-byte header per path and a 20-byte splat record
    # preallocated for every (vertex, path): linear in depth, 20/32 of the tape
    spl = [lib.lt_side_state_bytes(None, C.byref(_args(n, d, lt.RECORD_SPLATS))) for d in (8, 16, 32)]
    assert all(s == 16 * n + 20 * n * d for s, d in zip(spl, (8, 16, 32)))
    # the paper's card (16 GiB) cannot hold the depth-32 tape at 4M paths
    # plus its own working set while the replay records stay tiny
    assert tape[2] > 4 << 30 and res[2] < 256 << 20


def test_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert lib.lt_create(0, None, C.byref(h)) == lt.LT_ERR_ARG
    assert not h.value
    assert lib.lt_last_error(None) == b"null context"
