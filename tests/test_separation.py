"""The FP64 oracle and the HIP path share no code, and the product path has
no CPU fallback.

- The package, its C/HIP sources and the seeded input generators never
  import or include the oracle.
- The oracle never imports or includes the package.
- bench.py reaches the oracle only in its CPU-baseline leg, and
  __graft_entry__ only in build() (compiling the checker) and smoke().
- Importing the binding where the library has not been built raises
  ImportError instead of falling back to anything on the CPU.
"""
import ast
import glob
import os
import re
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2008_00216_amd")


def _imported_modules(tree):
    """(top-level module name, enclosing function name or None) per import."""
    out = []

    def visit(node, func):
        for child in ast.iter_child_nodes(node):
            f = func
            if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)):
                f = child.name if func is None else func
            if isinstance(child, ast.Import):
                out.extend((a.name.split(".")[0], f) for a in child.names)
            elif isinstance(child, ast.ImportFrom) and child.module and child.level == 0:
                out.append((child.module.split(".")[0], f))
            elif isinstance(child, ast.Call) and getattr(child.func, "attr", "") in (
                    "import_module", "spec_from_file_location"):
                for a in child.args:
                    if isinstance(a, ast.Constant) and isinstance(a.value, str):
                        out.append((a.value.split(".")[0], f))
            visit(child, f)

    visit(tree, None)
    return out


def _py_imports(path):
    with open(path) as fh:
        return _imported_modules(ast.parse(fh.read(), path))


def test_package_never_imports_the_oracle():
    files = glob.glob(os.path.join(PKG, "*.py")) + glob.glob(os.path.join(ROOT, "workloads", "*.py"))
    assert files
    for p in files:
        mods = {m for m, _ in _py_imports(p)}
        assert "oracle" not in mods, p


def test_oracle_never_imports_the_package():
    files = glob.glob(os.path.join(ROOT, "oracle", "*.py"))
    assert files
    for p in files:
        mods = {m for m, _ in _py_imports(p)}
        assert "paper_2008_00216_amd" not in mods, p
        assert "bench" not in mods, p


def test_c_sources_include_nothing_across_the_line():
    inc = re.compile(r'^\s*#\s*include\s*"([^"]+)"', re.M)
    for p in glob.glob(os.path.join(PKG, "csrc", "*")):
        for h in inc.findall(open(p).read()):
            assert "oracle" not in h, (p, h)
    for p in glob.glob(os.path.join(ROOT, "oracle", "*.c")) + glob.glob(os.path.join(ROOT, "oracle", "*.h")):
        text = open(p).read()
        for h in inc.findall(text):
            assert "csrc" not in h and "sv.h" not in h and "paper_2008_00216_amd" not in h, (p, h)


def test_bench_and_entry_reach_the_oracle_only_where_allowed():
    allowed = {"bench.py": {"cpu_baseline"}, "__graft_entry__.py": {"build", "smoke"}}
    for name, funcs in allowed.items():
        uses = [f for m, f in _py_imports(os.path.join(ROOT, name)) if m == "oracle"]
        assert uses, name
        assert all(f in funcs for f in uses), (name, uses)


def test_binding_without_library_raises(tmp_path):
    pkg = tmp_path / "paper_2008_00216_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(PKG, "__init__.py"), pkg / "__init__.py")
    code = ("import sys; sys.path.insert(0, sys.argv[1])\n"
            "try:\n"
            "    import paper_2008_00216_amd\n"
            "except ImportError as e:\n"
            "    print('IMPORTERROR', e)\n"
            "else:\n"
            "    print('IMPORTED')\n")
    r = subprocess.run([sys.executable, "-c", code, str(tmp_path)], cwd=str(tmp_path),
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "IMPORTERROR" in r.stdout and "is not built" in r.stdout, r.stdout
