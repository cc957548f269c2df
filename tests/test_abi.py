"""Host-side checks of the C ABI (no GPU needed): every function declared in
include/kb.h is exported by libkbatch.so, and the pure workspace-size query
answers without touching a device."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(kb_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def kb():
    import paper_2501_09398_amd as kb
    try:
        kb.lib()
    except ImportError as e:
        pytest.fail(f"libkbatch.so not built: {e}")
    return kb


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("kb_workspace_bytes", "kb_create", "kb_run", "kb_read", "kb_write",
                     "kb_reduce", "kb_last_timing", "kb_destroy", "kb_last_error",
                     "kb_set_option", "kb_kernels_per_iter", "kb_abi_version"):
        assert required in names


def test_every_declared_symbol_is_exported(kb):
    L = kb.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert L.kb_abi_version() == 1


def test_workspace_bytes_host_only(kb):
    n2 = kb.workspace_bytes(kb.HEAT2D, (256, 256))
    assert n2 >= 3 * 256 * 256 * 4
    assert n2 % 256 == 0
    assert kb.workspace_bytes(kb.HEAT3D, (8, 512, 512)) >= 2 * 8 * 512 * 512 * 4 + 512 * 512 * 4
    assert kb.workspace_bytes(kb.SKELETON, (1 << 16,)) >= (1 << 16) * 4
    assert kb.workspace_bytes(kb.FDTD3D, (128,)) >= 6 * 129 ** 3 * 4
    assert kb.workspace_bytes(kb.HEAT2D_MULTI, (2, 64, 64, 100, 30)) >= 3 * (64 * 64 + 3000) * 4
    # invalid problems / shapes answer 0
    assert kb.workspace_bytes(99, (4, 4)) == 0
    assert kb.workspace_bytes(kb.HEAT2D, (0, 4)) == 0
    assert kb.workspace_bytes(kb.HEAT2D, (4,)) == 0
    assert kb.workspace_bytes(kb.FDTD3D, (3,)) == 0
    assert kb.workspace_bytes(kb.HEAT2D_MULTI, (2, 64, 64)) == 0


def test_last_error_starts_empty_or_text(kb):
    assert isinstance(kb.lib().kb_last_error(), bytes)


def test_binding_refuses_without_library(tmp_path, monkeypatch):
    import paper_2501_09398_amd as kb
    monkeypatch.setattr(kb, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(kb, "_lib", None)
    with pytest.raises(ImportError):
        kb.lib()
