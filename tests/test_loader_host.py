"""The product path has no CPU fallback: without the built library the loader
raises instead of returning anything (no GPU needed)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_missing_library_raises_import_error():
    code = ("from paper_1612_00746_amd import _lib as L\n"
            "try:\n"
            "    L.load('/nonexistent/libctqw.so')\n"
            "except ImportError as e:\n"
            "    print('RAISED', e)\n"
            "else:\n"
            "    print('LOADED')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("RAISED"), r.stdout
    assert "not built" in r.stdout
