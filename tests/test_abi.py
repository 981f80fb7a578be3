"""The C-ABI library loads on a machine without a GPU and exports every declared symbol;
the Python binding refuses to run without a GPU (no CPU fallback)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "redve.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(redve_\w+)\(", hdr, re.M)))


def test_header_declarations_match_binding():
    import paper_1805_02158_amd as P
    assert _declared() == sorted(P.EXPORTS)


def test_library_exports_every_declared_symbol():
    import paper_1805_02158_amd as P
    lib = P.load_library()
    missing = [s for s in _declared() if not hasattr(lib, s)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True).stdout
    for s in _declared():
        assert re.search(rf"\bT {s}$", out, re.M), s


def test_library_is_gfx950_only():
    import paper_1805_02158_amd as P
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", P.LIB_PATH], capture_output=True,
                         text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout
    assert not re.search(r"gfx9(0|4)\d", out.stdout.replace("gfx950", ""))


def test_no_cpu_fallback_without_gpu():
    import torch
    import paper_1805_02158_amd as P
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(P.RedveError):
        P.Restorer(0)


def test_product_does_not_import_oracle():
    """The product package and bench's timed path never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1805_02158_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "liboracle" not in src, f
