"""The library carries a hash of the sources it was built from, and the
Python binding refuses to load a library built from other sources (a source
edit without a rebuild fails loudly instead of testing a stale binary)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = "paper_2605_16684_amd"


def test_library_hash_matches_the_tree():
    from paper_2605_16684_amd import build, esdg
    v = esdg.lib.esdg_version().decode()
    assert v.endswith("src:" + build.source_hash()), v
    names = [os.path.relpath(f, ROOT) for f in build.sources()]
    for must in ("esdg_api.hip", "esdg_device.hpp", "esdg_mixed.hpp", "esdg_curved.hpp", "esdg.h"):
        assert any(n.endswith(must) for n in names), (must, names)


def _import_in(root):
    code = f"import sys; sys.path.insert(0, {root!r}); import {PKG}.esdg"
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                          env={**os.environ, "PYTHONPATH": root})


def test_a_library_built_from_other_sources_is_refused(tmp_path):
    root = str(tmp_path)
    shutil.copytree(os.path.join(ROOT, PKG), os.path.join(root, PKG),
                    ignore=shutil.ignore_patterns("__pycache__", "*.tmp"))
    shutil.copytree(os.path.join(ROOT, "include"), os.path.join(root, "include"))
    ok = _import_in(root)
    assert ok.returncode == 0, ok.stderr
    with open(os.path.join(root, PKG, "csrc", "esdg_curved.hpp"), "a") as f:
        f.write("\n// edited after the build\n")
    bad = _import_in(root)
    assert bad.returncode != 0
    assert "built from other sources" in bad.stderr, bad.stderr[-2000:]
