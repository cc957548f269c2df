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
    if not os.path.exists(kb.LIB_PATH):
        # a fresh checkout: hipcc cross-compiles gfx950 without a GPU
        from paper_2501_09398_amd import build
        build.build()
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
    assert L.kb_abi_version() == 2


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


def header_defines():
    src = open(os.path.join(ROOT, "include", "kb.h")).read()
    return {k: int(v) for k, v in re.findall(r"#define\s+(KB_[A-Z0-9_]+)\s+(-?\d+)", src)}


def test_binding_constants_match_header(kb):
    d = header_defines()
    pairs = {"KB_OPT_REDUCE_EVERY": kb.OPT_REDUCE_EVERY, "KB_OPT_TILE": kb.OPT_TILE,
             "KB_OPT_GRAPH_UPDATE": kb.OPT_GRAPH_UPDATE, "KB_OPT_PERSISTENT": kb.OPT_PERSISTENT,
             "KB_OPT_SPIN_LIMIT": kb.OPT_SPIN_LIMIT,
             "KB_OPT_BUILDER": kb.OPT_BUILDER, "KB_OPT_TDEPTH": kb.OPT_TDEPTH,
             "KB_OPT_GRAPH_CACHE": kb.OPT_GRAPH_CACHE, "KB_OPT_MAX_NODES": kb.OPT_MAX_NODES,
             "KB_F_T": kb.F_T, "KB_F_P": kb.F_P, "KB_F_W": kb.F_W, "KB_F_SGSTATS": kb.F_SGSTATS,
             "KB_F_RESID": kb.F_RESID, "KB_F_REDLOG": kb.F_REDLOG, "KB_F_REDCOUNT": kb.F_REDCOUNT,
             "KB_HEAT2D": kb.HEAT2D, "KB_HEAT3D": kb.HEAT3D, "KB_SKELETON": kb.SKELETON,
             "KB_FDTD3D": kb.FDTD3D, "KB_HEAT2D_MULTI": kb.HEAT2D_MULTI,
             "KB_HEAT2D_SURROGATE": kb.HEAT2D_SURROGATE}
    for name, val in pairs.items():
        assert d[name] == val, name


def test_timing_struct_matches_header(kb):
    src = open(os.path.join(ROOT, "include", "kb.h")).read()
    body = re.search(r"typedef struct kb_timing \{(.*?)\} kb_timing;", src, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(double|int64_t)\s+([a-z_0-9]+);", body)
    assert [f for _, f in fields] == [f for f, _ in kb.Timing._fields_]
    import ctypes as C
    want = {"double": C.c_double, "int64_t": C.c_int64}
    assert [want[t] for t, _ in fields] == [t for _, t in kb.Timing._fields_]


def test_stream_probe_rejects_bad_arguments_without_a_gpu(kb):
    """Argument checks of the streaming calibration entry point happen
    before any HIP call."""
    import ctypes as C
    L = kb.lib()
    sec = C.c_double()
    buf = C.create_string_buffer(4096 + 256)
    aligned = (C.addressof(buf) + 255) // 256 * 256
    for nin, nout, n, ws, reps in ((0, 1, 64, 4096, 1), (1, 9, 64, 4096, 1), (1, 1, 6, 4096, 1),
                                   (2, 2, 1024, 4096, 1), (1, 1, 64, 4096, 0)):
        rc = L.kb_stream_probe(nin, nout, n, C.c_void_p(aligned), ws, None, reps, C.byref(sec))
        assert rc < 0, (nin, nout, n, ws, reps)
    rc = L.kb_stream_probe(1, 1, 64, C.c_void_p(aligned + 4), 4096, None, 1, C.byref(sec))
    assert rc == kb.EINVAL                            # misaligned workspace
