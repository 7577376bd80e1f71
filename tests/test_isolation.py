"""The product path (the HIP library and its Python binding) never reaches the
oracle and has no CPU fallback: checked on the sources and on the binding's
behaviour when the library is missing."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2512_16609_amd")


def _imports(path):
    tree = ast.parse(open(path).read(), filename=path)
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            yield from (a.name for a in node.names)
        elif isinstance(node, ast.ImportFrom):
            yield node.module or ""


def test_package_python_never_imports_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith(".py"):
                mods = list(_imports(os.path.join(dirpath, f)))
                assert not any(m == "oracle" or m.startswith("oracle.") for m in mods), (f, mods)


def test_native_sources_never_reference_the_oracle():
    csrc = os.path.join(PKG, "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        for line in text.splitlines():
            if line.lstrip().startswith("#include"):
                assert "oracle" not in line, (f, line)


def test_binding_fails_loudly_without_the_library():
    code = ("import paper_2512_16609_amd as h\n"
            "h.LIB_PATH = '/nonexistent/libhzd.so'\n"
            "h._lib = None\n"
            "try:\n"
            "    h.lib()\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n"
            "else:\n"
            "    raise SystemExit('no error')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "raised" in r.stdout, r.stdout + r.stderr
