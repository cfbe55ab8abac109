"""The C-ABI library loads on the CPU host and exports every entry point that
include/mgdelay.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgdelay.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(mgd_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_four_calls_of_the_boundary():
    names = _declared()
    for n in ("mgd_assemble_cells", "mgd_compress_stencils", "mgd_vcycle", "mgd_solve"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2005_03606_amd import binding
    assert os.path.exists(binding.library_path), "build first: python paper_2005_03606_amd/build.py"
    lib = ctypes.CDLL(binding.library_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", binding.library_path], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (mgd_\w+)", out))
    assert set(_declared()) <= exported


def test_binding_loads_and_reports_version():
    from paper_2005_03606_amd import binding
    assert binding.lib().mgd_version().startswith(b"mgdelay")


def test_header_is_valid_c():
    """The header compiles as plain C (no C++ or torch types)."""
    src = '#include "mgdelay.h"\nint main(void){return 0;}\n'
    p = subprocess.run(["gcc", "-x", "c", "-fsyntax-only", "-I", os.path.join(ROOT, "include"),
                        "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-"],
                       input=src, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr
