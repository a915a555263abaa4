"""Host-only checks of the C ABI: the library loads, exports every function include/sketch.h
declares, and validates configurations without touching a GPU."""
import ctypes
import os
import re

import pytest

import paper_1704_07669_amd as sk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "sketch.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sketch_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = sk.load_library()
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(sk.EXPORTED) == sorted(n for n in names if n in sk.EXPORTED)


def test_binding_has_c_names():
    for name in sk.EXPORTED:
        assert callable(getattr(sk, name))


def _cfg(**kw):
    base = dict(n=1000, m_capacity=2000, max_block_rows=200, k=10, l=20, b=10, compute=sk.F32,
                host_slots=0, host_src=sk.F32, want_u=0, omega_from_seed=1, seed=1)
    base.update(kw)
    return sk.sketch_config(**base)


def test_workspace_size_valid():
    n1 = sk.sketch_workspace_size(_cfg())
    n2 = sk.sketch_workspace_size(_cfg(m_capacity=4000))
    assert 0 < n1 < n2
    # host staging slots add max_block_rows x n x 4 bytes each
    n3 = sk.sketch_workspace_size(_cfg(host_slots=2))
    assert n3 - n1 >= 2 * 200 * 1000 * 4


@pytest.mark.parametrize("bad,msg", [
    (dict(n=0), "n must"),
    (dict(k=0), "k must"),
    (dict(k=30), "k must"),
    (dict(l=25, b=10), "b must"),
    (dict(b=33, l=66), "b must"),
    (dict(l=200, k=10), "l must"),
    (dict(n=10, l=20), "l must be <= n"),
    (dict(compute=9), "compute"),
    (dict(host_slots=1), "host_slots"),
    (dict(host_slots=2, compute=sk.F32, host_src=sk.BF16), "host_src"),
    (dict(m_capacity=0), "m_capacity"),
])
def test_workspace_size_rejects(bad, msg):
    with pytest.raises(sk.SketchError) as e:
        sk.sketch_workspace_size(_cfg(**bad))
    assert e.value.status == 1 and msg in str(e.value)


def test_init_rejects_without_touching_device():
    lib = sk.load_library()
    h = ctypes.c_void_p()
    cfg = _cfg()
    assert lib.sketch_init(ctypes.byref(h), ctypes.byref(cfg), None, 0, None) == 1
    assert b"workspace" in lib.sketch_last_error()
    # misaligned workspace
    assert lib.sketch_init(ctypes.byref(h), ctypes.byref(cfg), ctypes.c_void_p(16), 1 << 40,
                           None) == 1
    # too small
    assert lib.sketch_init(ctypes.byref(h), ctypes.byref(cfg), ctypes.c_void_p(256), 1024,
                           None) == 3
    # null handle everywhere
    assert lib.sketch_reset(None, 0) == 1
    assert lib.sketch_destroy(None) == 1


def test_config_struct_layout_matches_header(tmp_path):
    """The binding's ctypes structures against the C compiler's own layout of include/sketch.h
    (sizes and every field offset)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"sketch_config": sk.sketch_config, "sketch_server_config": sk.sketch_server_config,
               "sketch_server_stats": sk.sketch_server_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sketch.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    assert len(out.splitlines()) == sum(len(c._fields_) + 1 for c in structs.values())
    for line in out.splitlines():
        name, field, val = line.split()
        cls = structs[name]
        want = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(val) == want, (name, field)
