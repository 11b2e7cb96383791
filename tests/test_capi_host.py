"""CPU-side checks of the C-ABI library: it loads, exports every declared entry point, and
its Python binding mirrors the header's structs.  No compute call is made (no GPU here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hybro.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2402_18311_amd import hybro
    L = hybro.lib()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(hybro._SIGS) | {"hp_last_error"}


def test_binding_struct_layouts_match_header():
    from paper_2402_18311_amd import hybro
    # hp_die: 2 doubles, 2 int32, 1 double, 2 int32 -> 40 bytes with alignment
    assert C.sizeof(hybro.hp_die) == 40
    assert C.sizeof(hybro.hp_shape) == 16
    assert C.sizeof(hybro.hp_eval_params) == 24
    assert C.sizeof(hybro.hp_slot_state) == 80  # 3 int64, 6 doubles, 1 int64


def test_null_context_is_rejected_without_gpu():
    from paper_2402_18311_amd import hybro
    L = hybro.lib()
    assert L.hp_nesterov_step(None, None, 0) == hybro.HP_EINVAL
    assert L.hp_slot_bytes(None, None, None) == 0
    assert b"ctx" in L.hp_last_error() or L.hp_last_error() is not None


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2402_18311_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"(import\s+oracle|from\s+oracle|liborc|orc_)", txt), f


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2402_18311_amd import hybro
    monkeypatch.setattr(hybro, "_lib", None)
    monkeypatch.setattr(hybro, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        hybro.lib()


def test_header_is_plain_c_and_sizes_match_binding(tmp_path):
    """include/hybro.h compiles as pedantic C99 on its own, and its struct sizes are the
    binding's."""
    import shutil
    import subprocess
    from paper_2402_18311_amd import hybro
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "h.c"
    src.write_text('#include <stdio.h>\n#include "hybro.h"\nint main(void) {\n'
                   '  printf("%zu %zu %zu %zu %zu\\n", sizeof(hp_die), sizeof(hp_shape),\n'
                   '         sizeof(hp_eval_params), sizeof(hp_slot_state), sizeof(hp_iter_params));\n'
                   '  return 0;\n}\n')
    exe = tmp_path / "h"
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                        os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    sizes = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                            check=True).stdout.split()]
    assert sizes == [C.sizeof(hybro.hp_die), C.sizeof(hybro.hp_shape),
                     C.sizeof(hybro.hp_eval_params), C.sizeof(hybro.hp_slot_state),
                     C.sizeof(hybro.hp_iter_params)]
