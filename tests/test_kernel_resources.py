"""Every compiled kernel keeps its working set in registers: no scratch
(private memory) spills. The build records the compiler's per-kernel resource
report; a spill there means a variant's depth cap is too deep."""
import os
import re

import pytest

REPORT = os.path.join(os.path.dirname(__file__), "..", "paper_2305_07390_amd", "_build",
                      "kernel_resources.txt")


def test_no_kernel_spills_to_scratch():
    if not os.path.exists(REPORT):
        pytest.skip("library not built here (no resource report)")
    lines = [l for l in open(REPORT).read().splitlines() if l.strip()]
    assert lines, "empty resource report"
    spills = [l for l in lines if not re.search(r"scratch=0\b", l)]
    assert not spills, "kernels using scratch:\n" + "\n".join(spills)
