"""The documented build entry point works on a clean tree.

The files the repository would commit (tracked plus untracked-but-not-ignored,
so no built library and no build folder) are copied into a temporary
directory; there __graft_entry__.build() must compile libadct16.so from the
sources alone, import the package and find every symbol that
include/adct16.h declares.  hipcc cross-compiles for gfx950 without a GPU.
"""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _source_files():
    r = subprocess.run(["git", "ls-files", "--cached", "--others", "--exclude-standard", "-z"],
                       cwd=ROOT, capture_output=True)
    if r.returncode != 0:
        pytest.skip("not a git checkout")
    return [f for f in r.stdout.decode().split("\0") if f and os.path.isfile(os.path.join(ROOT, f))]


def _declared_symbols():
    with open(os.path.join(ROOT, "include", "adct16.h")) as f:
        text = f.read()
    names = re.findall(r"^\s*(?:adct16_status|const char\s*\*)\s*(adct16_\w+)\s*\(", text, re.M)
    assert len(names) >= 20
    return sorted(set(names))


@pytest.mark.skipif(not os.path.isdir(os.path.join(ROOT, ".git")), reason="needs the git checkout")
@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="needs hipcc")
def test_build_from_clean_tree(tmp_path):
    dst = tmp_path / "tree"
    for rel in _source_files():
        if rel.endswith(".so"):
            continue
        os.makedirs(dst / os.path.dirname(rel), exist_ok=True)
        shutil.copy2(os.path.join(ROOT, rel), dst / rel)
    pkg = dst / "paper_1606_05562_amd"
    assert not (pkg / "libadct16.so").exists()
    assert not (pkg / "_build").exists()
    syms = _declared_symbols()
    code = (
        "import ctypes, sys\n"
        "import __graft_entry__ as g\n"
        "g.build()\n"
        "import paper_1606_05562_amd as A\n"
        "lib = A.lib()\n"
        f"missing = [s for s in {syms!r} if not hasattr(lib, s)]\n"
        "assert not missing, missing\n"
        "assert A.lib()._name.startswith(sys.argv[1]), A.lib()._name\n"
        "print('clean build ok', len(missing))\n"
    )
    env = dict(os.environ)
    env.pop("PYTHONPATH", None)
    r = subprocess.run([sys.executable, "-c", code, str(dst)], cwd=dst, env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "clean build ok" in r.stdout
    assert (pkg / "libadct16.so").exists()
