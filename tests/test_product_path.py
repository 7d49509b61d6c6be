"""Host-only checks of the product path's independence from the test oracle
and of the absence of a CPU fallback."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1609_08094_amd")


def _sources(top, exts):
    for d, _, files in os.walk(top):
        if "__pycache__" in d or "_build" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_package_never_imports_the_oracle():
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle\b)", re.M)
    for f in _sources(PKG, (".py",)):
        assert not pat.search(open(f).read()), f


def test_kernels_and_oracle_share_no_sources():
    inc = re.compile(r'#include\s+"([^"]+)"')
    for f in _sources(os.path.join(PKG, "csrc"), (".hip", ".hpp", ".cpp")):
        for name in inc.findall(open(f).read()):
            assert "oracle" not in name, (f, name)
    for f in _sources(os.path.join(ROOT, "oracle"), (".py",)):
        assert "paper_1609_08094_amd" not in open(f).read(), f


def test_missing_library_raises_instead_of_falling_back():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1609_08094_amd import ccsdt\n"
            "try:\n"
            "    ccsdt.load_library('/nonexistent/libccsdt.so')\n"
            "except ImportError:\n"
            "    print('raised')\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.stdout.strip() == "raised", r.stdout + r.stderr
