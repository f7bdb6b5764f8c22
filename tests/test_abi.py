"""The C-ABI library loads and exports every entry point the header declares (no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kde_bw.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*(kde_[A-Za-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_selector_calls():
    names = declared_functions()
    for must in ("kde_bw_rot", "kde_bw_plugin", "kde_bw_lscv", "kde_lscv_curve", "kde_ctx_create"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1505_01998_amd as kde

    lib = ctypes.CDLL(kde.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(kde.EXPORTS) == set(declared_functions())


def test_binding_names_match_the_abi():
    import paper_1505_01998_amd as kde

    for name in declared_functions():
        assert callable(getattr(kde, name)), name


def test_library_has_gfx950_code_object():
    import paper_1505_01998_amd as kde

    blob = open(kde.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """Importing the binding without the built library raises instead of falling back."""
    import importlib.util

    pkg_dir = os.path.join(ROOT, "paper_1505_01998_amd")
    fake = tmp_path / "paper_1505_01998_amd"
    fake.mkdir()
    (fake / "__init__.py").write_text(open(os.path.join(pkg_dir, "__init__.py")).read())
    spec = importlib.util.spec_from_file_location("kde_nolib", str(fake / "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    try:
        spec.loader.exec_module(mod)
    except ImportError as e:
        assert "not built" in str(e)
    else:
        raise AssertionError("binding imported without its library")
