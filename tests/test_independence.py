"""Static checks that the oracle and the product path share no code."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = "paper_1905_00444_amd"


def _imports(path):
    tree = ast.parse(open(path).read())
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield a.name
        elif isinstance(node, ast.ImportFrom):
            yield (node.module or "")


def _py_files(d):
    for base, _, files in os.walk(os.path.join(ROOT, d)):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(base, f)


def test_oracle_imports_nothing_from_product():
    for f in _py_files("oracle"):
        for m in _imports(f):
            assert not m.startswith(PKG), (f, m)


def test_product_never_imports_oracle():
    for f in list(_py_files(PKG)):
        for m in _imports(f):
            assert not m.startswith("oracle"), (f, m)


def test_workloads_hold_no_product_or_oracle_imports():
    for f in _py_files("workloads"):
        for m in _imports(f):
            assert not m.startswith(PKG) and not m.startswith("oracle"), (f, m)


def test_native_sources_do_not_reference_oracle():
    csrc = os.path.join(ROOT, PKG, "csrc")
    if not os.path.isdir(csrc):
        return
    for base, _, files in os.walk(csrc):
        for f in files:
            src = open(os.path.join(base, f), errors="ignore").read()
            assert "oracle/" not in src and "import oracle" not in src, f
