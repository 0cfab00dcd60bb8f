"""The C ABI on the host: the library loads, exports every declared symbol, and
rejects invalid arguments before touching the device (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_1510_06340_amd import mf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mf.LIB_PATH):
        pytest.fail("libmf.so is not built (python -m paper_1510_06340_amd.build)")
    return mf.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(mf.EXPORTS)


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the ABI structs have the C compiler's size and field offsets."""
    import subprocess
    checks = {"mf_grid_desc": mf.GridDesc, "mf_stats": mf.Stats, "mf_surrogate": mf.Surrogate}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mf.h"', "int main(void) {"]
    for cname, cls in checks.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = []
    for cls in checks.values():
        want.append(C.sizeof(cls))
        want += [getattr(cls, f).offset for f, _ in cls._fields_]
    assert got == want


def _init(lib, desc, ptrs=None):
    h = C.c_void_p()
    arr = (C.c_void_p * 4)(*(ptrs or [1, 2, 3, 4]))
    return lib.mf_grid_init(C.byref(h), C.byref(desc), 1, arr, None), h


@pytest.mark.parametrize("field,value", [
    ("n", (0, 4, 4)), ("n", (65536, 65536, 2)), ("dx", (0.1, 0.0, 0.1)), ("dx", (0.1, float("nan"), 0.1)),
    ("bc", (0, 2, 0)), ("origin", (0.0, float("inf"), 0.0)), ("dtype", 7), ("limiter", 9), ("musta_k", 0),
    ("musta_k", 65), ("rk_order", 4), ("alpha", -1.0), ("flags", 16)])
def test_invalid_descriptors_are_rejected(lib, field, value):
    d = mf.make_desc((4, 4, 4), (0.1, 0.1, 0.1), (0, 0, 0), (0, 0, 0))
    if isinstance(value, tuple):
        getattr(d, field)[:] = list(value)
    else:
        setattr(d, field, value)
    rc, h = _init(lib, d)
    assert rc == mf.MF_ERR_ARG and not h.value
    assert len(mf.last_error()) > 0


def test_charge_descriptors_are_checked(lib):
    """MF_FLAG_CHARGE: five pointers per event, FP64 only, not with the unsplit ablation, and all
    events of a handle alike (checked before any device work)."""
    h = C.c_void_p()
    d = mf.make_desc((4, 4, 4), (0.1, 0.1, 0.1), (0, 0, 0), (0, 0, 0), flags=mf.MF_FLAG_CHARGE)
    arr5 = (C.c_void_p * 5)(1, 2, 3, 4, 0)
    assert lib.mf_grid_init(C.byref(h), C.byref(d), 1, arr5, None) == mf.MF_ERR_ARG
    assert "null state pointer" in mf.last_error()
    arr5 = (C.c_void_p * 5)(1, 2, 3, 4, 5)
    for bad in (dict(dtype=mf.MF_F32), dict(flags=mf.MF_FLAG_CHARGE | mf.MF_FLAG_UNSPLIT_HANCOCK)):
        db = mf.make_desc((4, 4, 4), (0.1, 0.1, 0.1), (0, 0, 0), (0, 0, 0), **dict(dict(flags=mf.MF_FLAG_CHARGE), **bad))
        assert lib.mf_grid_init(C.byref(h), C.byref(db), 1, arr5, None) == mf.MF_ERR_ARG
        assert not h.value
    two = (mf.GridDesc * 2)(d, mf.make_desc((4, 4, 4), (0.1, 0.1, 0.1), (0, 0, 0), (0, 0, 0)))
    arr10 = (C.c_void_p * 10)(*range(1, 11))
    assert lib.mf_grid_init(C.byref(h), two, 2, arr10, None) == mf.MF_ERR_ARG
    assert "charge" in mf.last_error()


def test_no_events_is_rejected(lib):
    d = mf.make_desc((4, 4, 4), (0.1, 0.1, 0.1), (0, 0, 0), (0, 0, 0))
    h = C.c_void_p()
    arr = (C.c_void_p * 4)(1, 2, 3, 4)
    assert lib.mf_grid_init(C.byref(h), C.byref(d), 0, arr, None) == mf.MF_ERR_ARG
    assert not h.value and "n_events" in mf.last_error()


def test_null_arguments_are_rejected(lib):
    d = mf.make_desc((4, 4, 4), (0.1, 0.1, 0.1), (0, 0, 0), (0, 0, 0))
    rc, _ = _init(lib, d, [1, 0, 3, 4])
    assert rc == mf.MF_ERR_ARG
    assert lib.mf_step(None, 0.1, 1, None) == mf.MF_ERR_ARG
    assert lib.mf_set_eos(None, 0, 0.3, None, None, 0, None) == mf.MF_ERR_ARG
    assert lib.mf_grid_free(None) == mf.MF_ERR_ARG
    assert lib.mf_totals(None, 0, None) == mf.MF_ERR_ARG
    assert "null" in mf.last_error()
