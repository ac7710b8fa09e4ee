"""The oracle and the HIP path share no code: neither side imports, includes
or links the other; the seeded input generators, the one module both use,
import neither; and the binding fails loudly when its library is missing
(there is no CPU fallback on the product path)."""
import ast
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2106_11143_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _files(d, exts):
    for dp, dn, fn in os.walk(d):
        dn[:] = [x for x in dn if x not in ("_build", "__pycache__")]
        for f in sorted(fn):
            if f.endswith(exts):
                yield os.path.join(dp, f)


def _imports(path):
    """Top-level names of every module a Python file imports (relative
    imports as '.name')."""
    out = set()
    for node in ast.walk(ast.parse(open(path).read(), path)):
        if isinstance(node, ast.Import):
            out |= {a.name.split(".")[0] for a in node.names}
        elif isinstance(node, ast.ImportFrom):
            out.add("." * node.level + (node.module or "").split(".")[0])
    return out


def _includes(path):
    return re.findall(r'^\s*#\s*include\s*[<"]([^>"]+)[>"]', open(path).read(), re.M)


def test_product_never_imports_or_includes_the_oracle():
    py = list(_files(PKG, (".py",)))
    assert len(py) >= 5
    for f in py:
        assert "oracle" not in _imports(f), f
    src = list(_files(os.path.join(PKG, "csrc"), (".hip", ".hpp", ".h", ".cpp"))) + list(_files(
        os.path.join(ROOT, "include"), (".h",)))
    assert len(src) >= 10
    for f in src:
        for inc in _includes(f):
            assert "oracle" not in inc, (f, inc)


def test_oracle_never_imports_includes_or_links_the_product():
    for f in _files(ORACLE, (".py",)):
        assert not (_imports(f) & {"paper_2106_11143_amd", "torch", ".api", ".inputs"}), f
    c = list(_files(ORACLE, (".c", ".h")))
    assert len(c) >= 2
    for f in c:
        for inc in _includes(f):
            assert os.path.basename(inc) != "coulomb.h" and "csrc" not in inc, (f, inc)
        assert "libcoulomb_mi355x" not in open(f).read(), f
    # the oracle's build links only the C library and libm
    assert "libcoulomb_mi355x" not in open(os.path.join(ORACLE, "oracle.py")).read()


def test_shared_generators_import_neither_side():
    mods = _imports(os.path.join(PKG, "inputs.py"))
    assert not mods & {"oracle", "torch", "ctypes", ".api", ".autograd", ".drivers", "."}, mods


def test_binding_fails_loudly_without_its_library():
    code = ("import paper_2106_11143_amd.api as A\n"
            "A.LIB_PATH = '/nonexistent/libcoulomb_mi355x.so'\n"
            "try:\n    A.lib()\nexcept RuntimeError as e:\n    print('raised:', e)\n"
            "else:\n    raise SystemExit('lib() returned without its library')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "raised:" in r.stdout and "not built" in r.stdout, r.stdout + r.stderr
