"""C-ABI library: loads on the CPU host and exports every symbol include/tda.h declares."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tda.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tda_[a-z_]+)\s*\(", text)))


def test_header_declarations_are_exported():
    import paper_2603_06010_amd as tda
    if not os.path.exists(tda.LIB_PATH):
        pytest.skip("library not built")
    nm = subprocess.run(["nm", "-D", "--defined-only", tda.LIB_PATH], capture_output=True,
                        text=True).stdout
    exported = set(re.findall(r" T (tda_\w+)", nm))
    missing = [f for f in _declared() if f not in exported]
    assert not missing, missing


def test_library_loads_and_reports_no_device():
    import numpy as np
    import paper_2603_06010_amd as tda
    if not os.path.exists(tda.LIB_PATH):
        pytest.skip("library not built")
    L = tda.load_library()
    assert L.tda_status_str(2).startswith(b"TDA_ENOTSPD")
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(tda.TdaError) as e:
        tda.Handle(np.array([1.0, 0.1]), 2)
    assert e.value.name == "TDA_ENODEV"


def test_binding_declares_header_functions():
    import paper_2603_06010_amd as tda
    for f in _declared():
        assert f in tda.EXPORTED_SYMBOLS, f
