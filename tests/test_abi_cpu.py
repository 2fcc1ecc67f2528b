"""Host-side checks of the C ABI: the library loads, exports every declared symbol,
and validates descriptors without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sl_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2009_07340_amd import binding as B
    lib = ctypes.CDLL(B.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTED) == names


_C_SIZES = {"int32_t": 4, "uint32_t": 4, "int64_t": 8, "uint64_t": 8, "double": 8, "float": 4, "size_t": 8}


def _header_fields(name):
    """(field, bytes) of `typedef struct name {...} name;` in include/sl.h, in order."""
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "sl.h")).read(), flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), src, re.S).group(1)
    out = []
    for decl in body.split(";"):
        decl = " ".join(decl.split())
        if not decl:
            continue
        m = re.match(r"(?:const )?(\w+)\s*(\*?)\s*(.*)$", decl)
        assert m, decl
        base, ptr, names = m.groups()
        for d in names.split(","):        # several declarators share the type
            f = re.fullmatch(r"\s*(\w+)(?:\[(\d+)\])?\s*", d)
            assert f, decl
            out.append((f.group(1), 8 if ptr else _C_SIZES[base] * int(f.group(2) or 1)))
    return out


@pytest.mark.parametrize("name", ["sl_mesh_desc", "sl_diag_t", "sl_schedule_t"])
def test_binding_structs_follow_the_header(name):
    """Field order and sizes of the ctypes mirrors equal the C declarations."""
    from paper_2009_07340_amd import binding as B
    py = getattr(B, name)
    got = [(f, ctypes.sizeof(t)) for f, t in py._fields_]
    assert got == _header_fields(name)


def test_required_bytes_counts_state_and_tables():
    from paper_2009_07340_amd import binding as B
    d = B.make_desc(1, 256, order=12, samples=1024)
    nbytes = B.sl_required_bytes(d)
    assert nbytes >= 1024 * 256 * 12 * 8
    assert nbytes < 1024 * 256 * 12 * 8 * 1.1
    d2 = B.make_desc(2, 64, 64, order=8, samples=256)
    assert B.sl_required_bytes(d2) >= 256 * 4096 * 64 * 8


@pytest.mark.parametrize("kw,code", [
    (dict(dim=3, kx=4), -1), (dict(dim=1, kx=0), -1), (dict(dim=1, kx=4, order=1), -1),
    (dict(dim=1, kx=4, order=17), -1), (dict(dim=1, kx=4, samples=0), -1),
    (dict(dim=1, kx=4, box=(1.0, 0.0, 0.0, 1.0)), -1), (dict(dim=1, kx=4, precision=7), -1),
])
def test_invalid_descriptors_are_rejected_before_any_device_call(kw, code):
    from paper_2009_07340_amd import binding as B
    d = B.make_desc(**kw)
    with pytest.raises(B.SLError) as ei:
        B.sl_required_bytes(d)
    assert ei.value.code == code
    with pytest.raises(B.SLError) as ei:
        B.sl_init_mesh(d)
    assert ei.value.code == code
    assert B.sl_last_error()


def test_null_handle_calls_fail_cleanly():
    from paper_2009_07340_amd import binding as B
    for call in (lambda: B.sl_step(None, 1e-3, 1), lambda: B.sl_sync(None), lambda: B.sl_get_step(None)):
        with pytest.raises(B.SLError) as ei:
            call()
        assert ei.value.code == -1
    assert B._lib.sl_destroy(None) == 0


def test_schedule_and_batch_argument_checks_without_a_device():
    from paper_2009_07340_amd import binding as B
    with pytest.raises(B.SLError) as ei:
        B.sl_set_schedule(None, 1, 1, 0)
    assert ei.value.code == -1
    with pytest.raises(B.SLError):
        B.sl_get_schedule(None)
    with pytest.raises(B.SLError):
        B.sl_autotune(None, 1e-3, 2)
    B.sl_step_batch([], [], 1)          # an empty batch is a no-op
    with pytest.raises(B.SLError):
        B.sl_step_batch([None], [1e-3], 1)


@pytest.mark.parametrize("fault", ["alloc", "host"])
def test_injected_allocation_failure_returns_enomem(monkeypatch, fault):
    """SL_FAULT makes the library's own allocations fail: creating a handle that
    needs them returns SL_ENOMEM and leaves no handle behind (no device call is
    made before the allocation, so this runs without a GPU)."""
    from paper_2009_07340_amd import binding as B
    d = B.make_desc(1, 16, order=8, samples=4)
    monkeypatch.setenv("SL_FAULT", fault)
    for _ in range(3):                   # repeated failures leave nothing behind
        with pytest.raises(B.SLError) as ei:
            B.sl_init_mesh(d)
        assert ei.value.code == B.SL_ENOMEM
        assert "fail" in B.sl_last_error()


def test_allocation_free_mean_checks_its_arguments_without_a_device():
    from paper_2009_07340_amd import binding as B
    for args in [(None, 4, 8, 1), (1, 4, 8, None), (1, 0, 8, 1), (1, 4, 0, 1), (1, 1 << 41, 8, 1),
                 (1, 1 << 30, 1 << 30, 1)]:
        with pytest.raises(B.SLError) as ei:
            B.sl_mean_noalloc(*args)
        assert ei.value.code == B.SL_EINVAL
