"""The C-ABI library loads without a GPU and exports every entry point that
include/shapetrace.h declares; argument validation that happens before any
device call returns ST_ERR_INVALID_ARG with a message."""
import ctypes
import os
import re

import pytest

from paper_2012_03939_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "shapetrace.h")).read()
    return sorted(set(re.findall(r"\b(st_[a-z_]+)\s*\(", txt)))


def test_header_declares_binding_list():
    assert _declared() == sorted(B.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = B.load()
    for name in _declared():
        assert hasattr(L, name), name


def test_host_side_validation_without_gpu():
    L = B.load()
    assert L.st_version() == 1
    o = L.st_render_opts_default()
    assert o.flags == 15 and abs(o.edge_spp_ratio - 1.0) < 1e-7 and o.queue_capacity == 0
    # the last field of the options struct: the binding's layout matches the header's
    assert o.max_workspace_bytes == 0 and not o.path_mask and not o.edge_mask
    out = ctypes.c_void_p()
    rc = L.st_scene_create(None, 0, None, 0, None, None, 0, None, 0, 0, 0, None, ctypes.byref(out))
    assert rc == -1 and b"non-NULL" in L.st_last_error()
    assert L.st_render(None, None, 0, 1, 1, 0, None, None, None) == -1
    assert L.st_render_backward(None, None, 0, 1, 1, 0, None, None, None, None, None) == -1
    assert L.st_render_batch(None, 0, None, None, 0, 1, 1, 0, None, None, None) == -1
    assert L.st_check_errors(None, None) == -1
    L.st_scene_destroy(None)
