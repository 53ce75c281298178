"""The C-ABI library loads without a GPU and exports every entry point that
include/labfm.h declares (no compute calls here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "labfm.h")
LIB = os.path.join(ROOT, "paper_1912_06441_amd", "liblabfm.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(labfm_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1912_06441_amd import build

        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("labfm_build_neighbours", "labfm_weights", "labfm_apply_operator", "labfm_step",
              "labfm_create", "labfm_destroy", "labfm_last_error", "labfm_combine"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (labfm_[a-z_0-9]+)", out))
    assert set(declared()) <= exported


def test_binding_names_match_header():
    import paper_1912_06441_amd as L

    assert sorted(L.EXPORTED) == declared()


def test_last_error_on_bad_arguments(lib):
    # argument validation runs before any device work
    lib.labfm_last_error.restype = ctypes.c_char_p
    lib.labfm_apply_operator.restype = ctypes.c_int
    rc = lib.labfm_apply_operator(None, None, None, ctypes.c_int64(0), ctypes.c_int64(0), 1, None, 0, None, None, None)
    assert rc == -1
    assert b"ctx" in lib.labfm_last_error()


def test_new_entry_points_validate_before_device_work(lib):
    """Batched weights, autotune query, the Burgers step and the warm-start calls
    reject a NULL context (or network) with LABFM_EINVAL and a message, without
    a GPU."""
    c = ctypes
    lib.labfm_last_error.restype = c.c_char_p
    calls = {
        "labfm_weights_batched": (None, 1, None, None, 0, None),
        "labfm_autotune_query": (None, 0, 0, c.c_uint(7), 8, None, None, None, None),
        "labfm_mlp_features": (None, None, None, c.c_int64(0), None, None, None, None, 64, None, None),
        "labfm_mlp_forward": (None, None, None, c.c_int64(0), None, None, 0, None),
        "labfm_mlp_backward": (None, None, None, None, None, c.c_int64(0), None, None),
        "labfm_mlp_moment_loss": (None, None, None, None, None, 8, c.c_uint(7), c.c_int64(0), None, None, None),
        "labfm_mlp_adam": (None, None, None, None, None, None, c.c_int64(0), None, c.c_int64(1), None),
        "labfm_mlp_cast_bf16": (None, None, None, c.c_int64(0), None),
        "labfm_burgers_step": (None, None, None, None, None, 1, 1, None),
        "labfm_poisson_solve": (None, None, None, None, None, None, None, None, None),
        "labfm_ns_step": (None, None, None, None, None, 1, None, None, None),
        "labfm_build_neighbours3": (None, None, None, None, c.c_int64(0), None, None, None, None, None, None),
        "labfm_weights3": (None, None, None, None, c.c_int64(0), None, None, 4, None, None, c.c_int64(0), None,
                           None, None, None, None, None),
    }
    for name, args in calls.items():
        fn = getattr(lib, name)
        fn.restype = c.c_int
        assert fn(*args) == -1, name
        assert lib.labfm_last_error(), name
    lib.labfm_mlp_cache_floats.restype = c.c_int64
    assert lib.labfm_mlp_cache_floats(None, c.c_int64(10)) == -1


def test_missing_library_fails_loudly():
    """Without the built library the binding raises; there is no other path."""
    code = ("import paper_1912_06441_amd as L\n"
            "try:\n"
            "    L.load_library('/nonexistent/liblabfm.so')\n"
            "except L.LabfmError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    raise SystemExit('loaded a library that does not exist')\n")
    r = subprocess.run([os.sys.executable, "-c", code], capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    assert "raised:" in r.stdout and "not built" in r.stdout
