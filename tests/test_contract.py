"""Contract checks that need no GPU.

* The product package never reaches the oracle: no module of
  paper_1810_05231_amd imports or names it, and importing the package (which
  loads libproxsdp) leaves `oracle` out of sys.modules.
* bench.py measures one GPU and says so for any other count, before touching
  a device.
"""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1810_05231_amd")


def test_package_sources_do_not_import_the_oracle():
    for name in sorted(os.listdir(PKG)):
        if not name.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(PKG, name)).read())
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                assert all(not a.name.split(".")[0] == "oracle" for a in node.names), name
            if isinstance(node, ast.ImportFrom):
                assert (node.module or "").split(".")[0] != "oracle", name


def test_importing_the_package_does_not_load_the_oracle():
    code = ("import sys; import paper_1810_05231_amd as p; "
            "from paper_1810_05231_amd._lib import lib; "
            "assert 'oracle' not in sys.modules, sorted(m for m in sys.modules if 'oracle' in m); "
            "print('ok')")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().endswith("ok")


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True,
                         text=True, timeout=600)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
