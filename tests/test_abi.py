"""The C ABI library loads and exports every function include/mechstep.h
declares; host-side argument checks reject bad calls before any device work.
Runs without a GPU: no call here reaches a kernel launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mechstep.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ms_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2105_00039_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build(force=False)
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_2105_00039_amd import _lib
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


def test_workspace_bytes_is_host_only(lib):
    from paper_2105_00039_amd import _lib
    a = lib.ms_workspace_bytes(1000, 5000, 1, _lib.MS_F32)
    b = lib.ms_workspace_bytes(1000, 5000, 1, _lib.MS_F64)
    c = lib.ms_workspace_bytes(2000, 5000, 1, _lib.MS_F32)
    assert 0 < a < b and a < c
    assert a % 256 == 0
    assert lib.ms_workspace_bytes(-1, 10, 1, _lib.MS_F32) == 0
    assert lib.ms_workspace_bytes(10, 10, 0, _lib.MS_F32) == 0


def test_host_validation_errors(lib):
    from paper_2105_00039_amd import _lib
    ws = _lib.ms_workspace()
    # null workspace / buffer
    assert lib.ms_workspace_init(None, ctypes.c_void_p(256), 1 << 20, 10, 10, 1, 0, None) == _lib.MS_EINVAL
    assert b"null" in lib.ms_last_error()
    assert lib.ms_workspace_init(ctypes.byref(ws), None, 1 << 20, 10, 10, 1, 0, None) == _lib.MS_EINVAL
    # misaligned buffer
    assert lib.ms_workspace_init(ctypes.byref(ws), ctypes.c_void_p(8), 1 << 20, 10, 10, 1, 0, None) == _lib.MS_EINVAL
    assert b"aligned" in lib.ms_last_error()
    # too small
    assert lib.ms_workspace_init(ctypes.byref(ws), ctypes.c_void_p(256), 64, 10, 10, 1, 0, None) == _lib.MS_EINVAL
    # bad dtype / capacities
    assert lib.ms_workspace_init(ctypes.byref(ws), ctypes.c_void_p(256), 1 << 20, 10, 10, 1, 7, None) == _lib.MS_EINVAL
    assert lib.ms_workspace_init(ctypes.byref(ws), ctypes.c_void_p(256), 1 << 40, 1 << 31, 10, 1, 0, None) == _lib.MS_ECAPACITY
    # step calls on a workspace without a buffer
    p = _lib.ms_params(2, 1, 0.01, 3, 0)
    assert lib.ms_grid_build(None, None, None, None, None, 10, 0.0, None) == _lib.MS_EINVAL
    assert lib.ms_mech_step(ctypes.byref(ws), ctypes.byref(p), None, None, None, None) == _lib.MS_EINVAL
    # integrate / probe argument checks
    assert lib.ms_integrate(None, None, None, None, None, None, -1, 0, None) == _lib.MS_EINVAL
    assert lib.ms_integrate(None, None, None, None, None, None, 5, 9, None) == _lib.MS_EINVAL
    assert lib.ms_integrate(None, None, None, None, None, None, 5, 0, None) == _lib.MS_EINVAL
    assert lib.ms_copy_probe(ctypes.c_void_p(16), ctypes.c_void_p(32), 17, None) == _lib.MS_EINVAL


def test_box_capacity_limit(lib):
    """A build holds at most 2^25 boxes (8192 buckets of 4096 boxes in the
    two-level sort); larger capacities are refused before any device work."""
    from paper_2105_00039_amd import _lib, MAX_BOXES
    assert MAX_BOXES == 1 << 25
    assert lib.ms_workspace_bytes(1000, 1 << 25, 1, _lib.MS_F32) > 0
    assert lib.ms_workspace_bytes(1000, (1 << 25) + 1, 1, _lib.MS_F32) == 0
    ws = _lib.ms_workspace()
    for boxes in ((1 << 25) + 1, 1 << 29, (1 << 31) - 2):
        st = lib.ms_workspace_init(ctypes.byref(ws), ctypes.c_void_p(256), 1 << 45, 1000, boxes, 1,
                                   _lib.MS_F32, None)
        assert st == _lib.MS_ECAPACITY, boxes
        assert b"2^25" in lib.ms_last_error()


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the header structs have the C compiler's sizes and offsets."""
    import subprocess
    from paper_2105_00039_amd import _lib
    prog = tmp_path / "sizes.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "mechstep.h"\n'
        'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(ms_params),'
        ' sizeof(ms_grid_info), sizeof(ms_workspace), offsetof(ms_grid_info, n_boxes),'
        ' offsetof(ms_workspace, dtype), offsetof(ms_workspace, n_sims), offsetof(ms_workspace, built));'
        'return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(_lib.ms_params), ctypes.sizeof(_lib.ms_grid_info),
            ctypes.sizeof(_lib.ms_workspace), _lib.ms_grid_info.n_boxes.offset,
            _lib.ms_workspace.dtype.offset, _lib.ms_workspace.n_sims.offset,
            _lib.ms_workspace.built.offset]
    assert got == want


def test_workspace_struct_mirror_matches_header():
    """The ctypes mirror of ms_workspace lists the header's fields in order
    with the same widths (the layout is part of the boundary)."""
    from paper_2105_00039_amd import _lib
    text = open(HEADER).read()
    body = text[text.rindex("typedef struct {", 0, text.index("} ms_workspace;")):text.index("} ms_workspace;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    decl = re.findall(r"(void\*|size_t|int64_t|int32_t)\s+(\w+);", body)
    width = {"void*": 8, "size_t": 8, "int64_t": 8, "int32_t": 4}
    mirror = _lib.ms_workspace._fields_
    assert [n for _, n in decl] == [n for n, _ in mirror]
    for (ty, name), (_, cty) in zip(decl, mirror):
        assert ctypes.sizeof(cty) == width[ty], name
    # no padding between fields; the end is padded to the struct's 8-byte alignment
    offs = [getattr(_lib.ms_workspace, n).offset for _, n in decl]
    assert offs == [sum(width[t] for t, _ in decl[:i]) for i in range(len(decl))]
    assert ctypes.sizeof(_lib.ms_workspace) == (sum(width[t] for t, _ in decl) + 7) // 8 * 8


def test_header_is_plain_c99(tmp_path):
    """The boundary header compiles as C99 on its own (plain pointers and
    sizes, no HIP or torch types), so any C caller can use it."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "use_header.c"
    src.write_text('#include "mechstep.h"\n'
                   "int main(void) { ms_workspace w; ms_params p; ms_grid_info g;\n"
                   "  (void)w; (void)p; (void)g; return 0; }\n")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-fsyntax-only", "-I", os.path.dirname(HEADER), str(src)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """Without the built HIP library the package raises instead of falling
    back to anything else, and no product module reaches the oracle."""
    from paper_2105_00039_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libmechstep.so"))
    with pytest.raises(ImportError, match="no fallback"):
        _lib.load()
    pkg = os.path.join(ROOT, "paper_2105_00039_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liborc" not in text, f


def test_noalloc_host_checks(lib):
    """The step without allocation refuses more agents than its static
    workspace holds, and bad arguments, before touching the device; the
    header's limits are the binding's."""
    from paper_2105_00039_amd import _lib
    text = open(HEADER).read()
    assert f"#define MS_NOALLOC_MAX_AGENTS {_lib.NOALLOC_MAX_AGENTS}" in text
    assert f"#define MS_NOALLOC_MAX_BOXES {_lib.NOALLOC_MAX_BOXES}" in text
    p = _lib.ms_params(2, 1, 0.01, 3, 0)
    nul = ctypes.c_void_p(0)
    st = lib.ms_mech_step_noalloc(nul, nul, nul, nul, _lib.NOALLOC_MAX_AGENTS + 1, _lib.MS_F32, 0.0,
                                  ctypes.byref(p), nul, nul, nul, nul, nul)
    assert st == _lib.MS_ECAPACITY
    assert b"MS_NOALLOC_MAX_AGENTS" in lib.ms_last_error()
    assert lib.ms_mech_step_noalloc(nul, nul, nul, nul, -1, _lib.MS_F32, 0.0, ctypes.byref(p),
                                    nul, nul, nul, nul, nul) == _lib.MS_EINVAL
    assert lib.ms_mech_step_noalloc(nul, nul, nul, nul, 10, 9, 0.0, ctypes.byref(p),
                                    nul, nul, nul, nul, nul) == _lib.MS_EINVAL
    bad = _lib.ms_params(2, 1, -0.01, 3, 0)
    assert lib.ms_mech_step_noalloc(nul, nul, nul, nul, 10, _lib.MS_F32, 0.0, ctypes.byref(bad),
                                    nul, nul, nul, nul, nul) == _lib.MS_EINVAL
    assert lib.ms_mech_step_noalloc(nul, nul, nul, nul, 10, _lib.MS_F32, 0.0, ctypes.byref(p),
                                    nul, nul, nul, nul, nul) == _lib.MS_EINVAL
