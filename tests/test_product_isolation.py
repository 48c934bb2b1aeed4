"""The product path stands on the HIP library alone: its binding fails loudly
when libwv.so is missing, and no product source reaches the oracle, which
only the tests, the smoke check and the bench's CPU-baseline leg may use.
Host-only: no device is touched."""
import ast
import os
import re
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2208_10859_amd")


def test_binding_fails_loudly_without_library(tmp_path):
    dst = tmp_path / "paper_2208_10859_amd"
    dst.mkdir()
    for f in os.listdir(PKG):
        if f.endswith(".py"):
            shutil.copy(os.path.join(PKG, f), dst / f)
    assert not (dst / "libwv.so").exists()
    for mod in ("wv", "fmt", "cnn"):
        r = subprocess.run([sys.executable, "-c", f"import paper_2208_10859_amd.{mod}"],
                           cwd=tmp_path, env={**os.environ, "PYTHONPATH": str(tmp_path)},
                           capture_output=True, text=True, timeout=300)
        assert r.returncode != 0, mod
        assert "ImportError" in r.stderr and "libwv.so is missing" in r.stderr, (mod, r.stderr[-400:])


def _product_sources():
    for base in (PKG, os.path.join(ROOT, "include")):
        for dirpath, _, files in os.walk(base):
            for f in files:
                if f.endswith((".py", ".hip", ".cpp", ".h")):
                    yield os.path.join(dirpath, f)


def test_product_sources_do_not_reach_the_oracle():
    py_import = re.compile(r"^\s*(from\s+oracle\b|import\s+oracle\b|from\s+\.\.oracle\b)", re.M)
    c_include = re.compile(r'#\s*include\s*[<"][^>"]*oracle', re.M)
    seen = 0
    for path in _product_sources():
        txt = open(path, encoding="utf-8").read()
        assert not py_import.search(txt), f"{path} imports the oracle"
        assert not c_include.search(txt), f"{path} includes oracle code"
        assert "importlib" not in txt or "oracle" not in txt, path
        seen += 1
    assert seen > 10


def _oracle_import_owners(path):
    """Names of the top-level functions holding each oracle import of a module
    (None for an import at module level)."""
    tree = ast.parse(open(path, encoding="utf-8").read())
    owners = []

    def visit(node, owner):
        for child in ast.iter_child_nodes(node):
            o = owner
            if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) and owner is None:
                o = child.name
            if isinstance(child, ast.ImportFrom) and (child.module or "").split(".")[0] == "oracle":
                owners.append(owner)
            elif isinstance(child, ast.Import) and any(a.name.split(".")[0] == "oracle" for a in child.names):
                owners.append(owner)
            visit(child, o)

    visit(tree, None)
    return owners


def test_bench_and_entry_use_the_oracle_only_where_allowed():
    bench = _oracle_import_owners(os.path.join(ROOT, "bench.py"))
    assert bench and set(bench) == {"cpu_baseline"}, bench
    entry = _oracle_import_owners(os.path.join(ROOT, "__graft_entry__.py"))
    assert entry and set(entry) == {"smoke"}, entry
