"""Host-only checks of the two boundaries the parity claims rest on: the
product library and the oracle share no code, and the product path has no
fallback (the binding refuses to run without the HIP library)."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1511_07207_amd")
CSRC = os.path.join(PKG, "csrc")
ORACLE = os.path.join(ROOT, "oracle")


def _read(path):
    with open(path, encoding="utf-8") as f:
        return f.read()


def test_oracle_includes_only_system_headers():
    src = _read(os.path.join(ORACLE, "ks_oracle.c"))
    includes = re.findall(r'^\s*#\s*include\s*([<"][^>"]+[>"])', src, re.M)
    assert includes and all(i.startswith("<") for i in includes), includes
    # nothing of the library's headers or kernels by name
    assert "ks.h" not in src and "ks_internal" not in src and "ks_device" not in src


def test_library_sources_do_not_reach_the_oracle():
    for name in os.listdir(CSRC):
        src = _read(os.path.join(CSRC, name))
        assert "oracle" not in src.lower(), name
        for inc in re.findall(r'^\s*#\s*include\s*"([^"]+)"', src, re.M):
            assert os.path.exists(os.path.join(CSRC, inc)) or inc == "ks.h", (name, inc)
    for name in os.listdir(PKG):
        if name.endswith(".py"):
            src = _read(os.path.join(PKG, name))
            assert not re.search(r"^\s*(import|from)\s+oracle\b", src, re.M), name


def test_oracle_does_not_import_the_library():
    for name in os.listdir(ORACLE):
        if name.endswith(".py"):
            src = _read(os.path.join(ORACLE, name))
            assert "paper_1511_07207_amd" not in src, name


def test_binding_fails_loudly_without_the_hip_library():
    """With the library path pointing nowhere, the first call raises: there
    is no CPU route to a result."""
    code = (
        "import paper_1511_07207_amd._native as N\n"
        "N.LIB_PATH = '/nonexistent/libks.so'\n"
        "N._lib = None\n"
        "try:\n"
        "    N.lib()\n"
        "except RuntimeError as e:\n"
        "    print('raised', e)\n"
        "else:\n"
        "    print('loaded')\n"
    )
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=120)
    assert "raised" in out.stdout and "missing" in out.stdout, (out.stdout, out.stderr)
