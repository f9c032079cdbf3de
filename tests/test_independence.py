"""The oracle and the HIP library share no code: neither imports, includes or loads the other,
and the seeded input generators import neither (no GPU)."""
import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = "paper_1909_12234_amd"


def _files(folder, exts):
    for dirpath, _, names in os.walk(os.path.join(ROOT, folder)):
        if "__pycache__" in dirpath:
            continue
        for n in names:
            if n.endswith(exts):
                yield os.path.join(dirpath, n)


def _imported_modules(path):
    mods = set()
    for node in ast.walk(ast.parse(open(path).read())):
        if isinstance(node, ast.Import):
            mods.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.level == 0 and node.module:
            mods.add(node.module.split(".")[0])
    return mods


def test_oracle_imports_neither_the_library_nor_its_sources():
    for f in _files("oracle", (".py",)):
        assert PKG not in _imported_modules(f), f
    for f in _files("oracle", (".c", ".h")):
        src = open(f).read()
        assert not re.search(r'#include\s+"', src), f  # system headers only
        assert "lqtrace" not in src and PKG not in src, f


def test_library_never_reaches_the_oracle():
    for f in _files(PKG, (".py",)):
        assert "oracle" not in _imported_modules(f), f
        assert "liboracle" not in open(f).read(), f
    for f in list(_files(PKG, (".hip", ".h", ".cpp"))) + list(_files("include", (".h",))):
        src = open(f).read()
        assert "oracle" not in src.lower(), f


def test_input_generators_import_neither_side():
    for f in _files("synth", (".py",)):
        mods = _imported_modules(f)
        assert PKG not in mods and "oracle" not in mods, f
