"""The ablation runner's configuration (host only): every switch it sets is
one the kernel headers define with a default, every step names a known
variant, each sequence ends with the library itself, and the defaults are
the library's (all on, four planes)."""
import os
import re

from paper_2305_07390_amd import ablation

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2305_07390_amd", "csrc")


def _defaults():
    out = {}
    for name in ("tb2d_impl.hpp", "tb3d_impl.hpp"):
        text = open(os.path.join(CSRC, name)).read()
        for m in re.finditer(r"#ifndef (STENCIL_ABL_\w+)\s*\n#define \1 (\d+)", text):
            out[m.group(1)] = int(m.group(2))
    return out


def test_switches_exist_with_library_defaults():
    d = _defaults()
    assert d == {"STENCIL_ABL_PREFETCH": 1, "STENCIL_ABL_SCHED_BARRIER": 1, "STENCIL_ABL_SPLIT_BODY": 1,
                 "STENCIL_ABL_XCD_ORDER": 1, "STENCIL_ABL_PLANES": 4}
    for defs in ablation.VARIANTS.values():
        assert set(defs) <= set(d)
        # a variant turns switches off, never on beyond the library
        assert all(v <= d[k] for k, v in defs.items())


def test_steps_name_known_variants_and_end_with_the_library():
    for dim, steps in ablation.STEPS.items():
        assert steps[-1][2] is None, dim
        for name, what, variant, depth, flags in steps:
            assert variant is None or variant in ablation.VARIANTS
            assert depth >= 1 and what
    for src in ablation.ONLY:
        assert os.path.exists(os.path.join(CSRC, src))
