"""The product path and the oracle stay apart (CPU).

The package `paper_2109_10392_amd` never imports the oracle (only tests,
`smoke()` and bench.py's CPU baseline may), and without the built library every
entry point raises instead of computing anything on the host.
"""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2109_10392_amd")


def _imports(path):
    tree = ast.parse(open(path).read(), filename=path)
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield a.name
        elif isinstance(node, ast.ImportFrom):
            yield node.module or ""


def test_package_never_imports_the_oracle():
    for name in sorted(os.listdir(PKG)):
        if name.endswith(".py"):
            mods = list(_imports(os.path.join(PKG, name)))
            assert not any(m == "oracle" or m.startswith("oracle.") for m in mods), (name, mods)


def test_missing_library_raises():
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2109_10392_amd import traj as T\n"
        "T.LIB_PATH = '/nonexistent/libtraj.so'\n"
        "T._lib = None\n"
        "from paper_2109_10392_amd import scenes as S\n"
        "for call in (T.lib, lambda: T.Solver(S.DEFAULT_PARAMS, [(100, 10.0, 10)])):\n"
        "    try:\n"
        "        call()\n"
        "    except RuntimeError as e:\n"
        "        print('raised', e)\n"
        "    else:\n"
        "        print('ran')\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert out.stdout.count("raised") == 2 and "ran" not in out.stdout, out.stdout + out.stderr
